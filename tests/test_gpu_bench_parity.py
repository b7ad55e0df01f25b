"""Full-size GPU parity of what the benchmark times, built by the benchmark's
own setup functions (so the launches checked are the launches timed):

- the batched halo step: float64 512^3 array (1 GiB) in 4 rotating copies,
  12 faces (ghost widths 1 and 4) packed by one batched launch and unpacked
  into a zeroed copy by another, autotuned as the benchmark tunes it, then a
  persistent graph-replayed configuration and plain launches; after the
  warm-up and the timed steps every packed face of every copy and every
  unpacked array equal the oracle's;
- the 4096-request batch at its stated sizes (log-uniform 64 B..16 MiB over
  vector(2^21, 1, s), the 512^3 faces and the 1M-block hindexed layout in a
  2 GiB buffer): every request of the autotuned launch, of a persistent
  graph launch and of per-request kernels equals the oracle's partial pack;
- served requests of the serving trace at full size (Zipf sizes up to
  64 MiB, 500 resident types): a sample covering every type family, both
  directions and the largest requests, submitted in bursts so they batch and
  overlap on the device, each compared with the oracle (pack output; the
  whole destination span of an unpack, gaps included).
"""
import concurrent.futures as cf

import numpy as np
import pytest

from gpu_util import note
from oracle import build_type as obuild
from paper_2402_12274_amd import inputs

pytestmark = pytest.mark.gpu

MiB = 1 << 20
GiB = 1 << 30


@pytest.fixture(scope="module")
def env():
    from gpu_util import torch_cuda

    torch = torch_cuda()
    import bench
    from paper_2402_12274_amd import mdt

    return torch, mdt, bench


def _threads():
    import os

    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return 4


def test_halo_step_as_benched(env):
    torch, mdt, bench = env
    W = bench.workload("halo")
    stream = torch.cuda.current_stream()
    ms = mdt.Stream(stream.cuda_stream)
    note("halo step as benched: setup + autotune")
    S = bench.step_setup(torch, mdt, W, 4, True, ms)
    assert S["R"] == 4
    host = inputs.random_bytes(W["src_bytes"], seed=W["seed"])
    refs = []
    exp_dst = np.zeros_like(host)
    for label, spec, count in W["reqs"]:
        o = obuild(spec)
        p = o.pack(host, 0, count)
        o.unpack(p, exp_dst, 0, count)
        refs.append(p)
    del host
    exp_dev = torch.from_numpy(exp_dst).to("cuda")
    ref_dev = [torch.from_numpy(p).to("cuda") for p in refs]
    del exp_dst
    tuned = (S["batches"][0][0].get_config(), S["batches"][0][1].get_config())
    for name, cfgs, batched in (("autotuned", tuned, True),
                                ("persistent graph", (mdt.BatchConfig(1024, 4, 0, 1, 0),) * 2, True),
                                ("dynamic graph", (mdt.BatchConfig(4096, 8, 1, 1, 0),) * 2, True),
                                ("plain launches", None, False)):
        note(f"halo step as benched: {name}")
        for d in S["dsts"]:
            d.zero_()
        for ps in S["packed"]:
            for p in ps:
                p.fill_(0x5A)
        if batched:
            bench.set_step_config(S, *cfgs)
        bench.timed_steps(torch, S, batched, ms, stream, 8, 3, mdt)
        torch.cuda.synchronize()
        for r in range(S["R"]):
            for k, ref in enumerate(ref_dev):
                assert torch.equal(S["packed"][r][k][:ref.numel()], ref), (name, r, W["reqs"][k][0])
            assert torch.equal(S["dsts"][r], exp_dev), (name, r)


def test_batch4096_full_size(env):
    torch, mdt, bench = env
    stream = torch.cuda.current_stream()
    ms = mdt.Stream(stream.cuda_stream)
    note("batch4096 full size: setup")
    B = bench.batch4096_setup(torch, mdt)
    hosts = {k: inputs.random_bytes(b, seed=seed) for k, (b, seed) in bench.batch4096_arenas().items()}
    otypes = {}
    for r in B["reqs"]:
        if r["spec_key"] not in otypes:
            otypes[r["spec_key"]] = obuild(r["spec"] if r["spec"] is not None else B["hspec"])
    offs = B["offs"]
    exp = np.zeros(int(offs[-1]), np.uint8)
    kinds = set()

    def expect(i):
        r = B["reqs"][i]
        n = B["plan"][i][2]
        p = otypes[r["spec_key"]].pack(hosts[r["kind"]], 0, 1, 0, n)
        assert p.size == n
        exp[int(offs[i]):int(offs[i]) + n] = p
        return r["kind"], n

    note("batch4096 full size: oracle")
    with cf.ThreadPoolExecutor(_threads()) as ex:
        done = list(ex.map(expect, range(len(B["reqs"]))))
    for kind, n in done:
        kinds.add(kind)
    assert kinds == {"vector", "face", "hindexed"} and len(done) == 4096
    # the largest requests of each kind are in the mix at full size
    assert max(n for k, n in done if k == "vector") > 15 * MiB
    assert max(n for k, n in done if k == "hindexed") > 15 * MiB
    del hosts
    exp_dev = torch.from_numpy(exp).to("cuda")
    b = B["batch"]
    tuned = b.autotune(ms)
    for name, cfg in (("autotuned", tuned), ("persistent graph", mdt.BatchConfig(1024, 4, 0, 1, 0)),
                      ("per-request kernels", mdt.BatchConfig(1024, 0, 3, 0, 0))):
        note(f"batch4096 full size: {name} {mdt.config_dict(cfg)}")
        b.set_config(cfg)
        B["out"].fill_(0)
        for _ in range(2):
            b.launch(ms)
        torch.cuda.synchronize()
        if not torch.equal(B["out"], exp_dev):
            got = B["out"].cpu().numpy()
            bad = [i for i in range(4096)
                   if not np.array_equal(got[int(offs[i]):int(offs[i + 1])], exp[int(offs[i]):int(offs[i + 1])])]
            pytest.fail(f"{name}: {len(bad)} requests differ from the oracle, first {bad[:5]}")


def test_served_requests_full_size(env):
    torch, mdt, bench = env
    note("served requests at full size: setup")
    V = bench.serve_setup(torch, mdt)
    reqs, info = bench.serve_requests(V, 20000.0, 1.0)
    fam = info["fam"]
    hosts = {f: inputs.random_bytes(b, seed=inputs.DEFAULT_SEED + i)
             for i, (f, b) in enumerate(bench.SERVE_ARENAS.items())}
    pk_host = inputs.random_bytes(64 << 20, seed=5)
    # the sample: the largest packs, the largest unpacks whose span fits 1 GiB,
    # then requests of every (family, direction) pair
    pick = []
    for up in (0, 1):
        idx = np.nonzero((reqs["unpack"] == up) & (reqs["span"] <= GiB))[0]
        pick += list(idx[np.argsort(reqs["target"][idx])[-3:]])
    g = np.random.default_rng(11)
    for f in bench.SERVE_ARENAS:
        for up in (0, 1):
            idx = np.nonzero((fam == f) & (reqs["unpack"] == up) & (reqs["span"] <= 256 * MiB))[0]
            pick += list(g.choice(idx, size=min(5, idx.size), replace=False))
    pick = sorted(set(int(i) for i in pick))
    assert any(reqs["target"][i] > 32 * MiB for i in pick)
    srv = mdt.Server(nstreams=8, budget_bytes=32 << 30, max_batch=256, max_inflight=2)
    srv.start()
    otypes = {}
    checked = 0
    try:
        for w0 in range(0, len(pick), 12):
            wave = pick[w0:w0 + 12]
            note(f"served requests at full size: wave {w0 // 12} ({len(wave)} requests)")
            live = []
            for i in wave:
                q = reqs[i]
                t = V["types"][int(q["type_index"])]
                if q["unpack"]:
                    dst = torch.zeros(int(q["span"]), dtype=torch.uint8, device="cuda")
                    torch.cuda.synchronize()
                    h = srv.submit_unpack(int(q["packed"]), int(q["target"]), dst.data_ptr() + int(q["origin_off"]),
                                          int(q["count"]), t, 0)
                else:
                    dst = None
                    h = srv.submit_pack(int(q["typed"]), int(q["count"]), t, 0, int(q["target"]))
                live.append((i, h, dst))
            for i, h, dst in live:
                srv.wait(h)
                st, pk, nb, lat = srv.result(h)
                q = reqs[i]
                assert st == 0 and nb == int(q["target"]), (i, st, nb)
                if not q["unpack"]:
                    dst = torch.empty(max(1, nb), dtype=torch.uint8, device="cuda")
                    _hip_copy(dst.data_ptr(), pk, nb)
                srv.release(h)
                ti = int(q["type_index"])
                if ti not in otypes:
                    otypes[ti] = obuild(V["fam_types"][ti][1])
                o = otypes[ti]
                if q["unpack"]:
                    exp = np.zeros(int(q["span"]), np.uint8)
                    o.unpack(pk_host[:int(q["target"])], exp, int(q["origin_off"]), int(q["count"]), 0)
                else:
                    exp = o.pack(hosts[fam[i]], 0, int(q["count"]), 0, int(q["target"]))
                got = torch.from_numpy(exp).to("cuda")
                assert torch.equal(dst[:exp.size], got), (i, fam[i], "unpack" if q["unpack"] else "pack")
                checked += 1
    finally:
        srv.stop()
        srv.close()
    assert checked == len(pick)


def _hip_copy(dst, src, n):
    import ctypes

    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    assert hip.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), n, 3) == 0
