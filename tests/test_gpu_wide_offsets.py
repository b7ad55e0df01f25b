"""Byte addresses beyond 4 GiB on the GPU: layouts whose displacements, extents
and packed-stream offsets do not fit 32 bits, against the oracle.

One 5 GiB buffer holds, at once:
- an hvector of 3 vectors every 1.5 GiB + 8 B (extent 4.5 GiB);
- a resized vector of extent 2.25 GiB taken twice (count 2: the second
  element starts past 2^31);
- a hindexed of 2000 short blocks at permuted displacements over 5 GiB
  (the run-table path);
- a 5 GiB contiguous type, packed and unpacked in a 3 MiB window that starts
  4.25 GiB into the packed stream.

Each is flattened on the host and on the device, packed whole and in byte
windows (offset + budget), unpacked into a zeroed 5 GiB buffer that must
equal the oracle's unpack everywhere, and run as requests of one batch.
"""
import numpy as np
import pytest

from gpu_util import first_diff, note
from oracle import build_type as obuild
from paper_2402_12274_amd import inputs

pytestmark = pytest.mark.gpu

GiB = 1 << 30
MiB = 1 << 20
SPAN = 5 * GiB + MiB
D = inputs.DOUBLE


def _specs():
    g = inputs.rng(4242)
    n = 2000
    disps = np.sort(g.choice((5 * GiB - 4096) // 64, size=n, replace=False)) * 64
    lens = g.integers(1, 64, size=n)
    perm = g.permutation(n)
    hind = ("hindexed", [int(x) for x in lens[perm]], [int(x) for x in disps[perm]], inputs.BYTE)
    return [
        # name, spec, count, windows (inoffset, budget)
        ("wide", ("hvector", 4, 3, (3 << 29) + 8, ("vector", 1000, 2, 7, D)), 1,
         [(0, 4096), (95_999, 17), (100_000, 50_000), (191_990, -1)]),
        ("rec", ("resized", 0, 9 << 28, ("vector", 64, 1, 3, D)), 2, [(500, 24), (511, 2), (512, 300)]),
        ("hind", hind, 1, [(0, 1000), (32_000, 7), (60_000, -1)]),
        ("contig", ("contiguous", 5 << 27, D), 1, [((17 << 28) + 3, 3 * MiB + 5)]),
    ]


@pytest.fixture(scope="module")
def env():
    from gpu_util import torch_cuda

    torch = torch_cuda()
    from paper_2402_12274_amd import mdt

    cases = []
    host = np.zeros(SPAN, np.uint8)
    for k, (name, spec, count, wins) in enumerate(_specs()):
        o = obuild(spec)
        nseg, _ = o.iov_len(-1, count)
        if name == "contig":
            regions = [(lo - 4096, lo + n + 4096) for lo, n in wins]
        else:
            b, ln = o.iov(0, nseg, count)
            regions = [(int(x) - 128, int(x) + int(m) + 128) for x, m in zip(b, ln)]
        for i, (lo, hi) in enumerate(regions):
            lo, hi = max(0, lo), min(SPAN, hi)
            host[lo:hi] = inputs.random_bytes(hi - lo, seed=1000 * k + i % 997)
        cases.append((name, spec, count, wins, o, mdt.build_type(spec), nseg))
    dev = torch.from_numpy(host).to("cuda")
    memo = {}

    def opack(name, o, count, off, budget):
        # the oracle's pack, kept: it walks the contiguous layout element by element
        key = (name, count, off, budget)
        if key not in memo:
            memo[key] = o.pack(host, 0, count, off, budget)
        return memo[key]

    return torch, mdt, host, dev, cases, opack


def _chunks_equal(torch, dev, exp):
    # compares a device buffer with a host array 256 MiB at a time
    step = 256 * MiB
    for lo in range(0, exp.size, step):
        got = dev[lo:lo + step].cpu().numpy()
        d = first_diff(got, exp[lo:lo + step])
        if d is not None:
            return lo + d
    return None


def test_wide_flatten_host_and_device(env):
    torch, mdt, host, dev, cases, opack = env
    s = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    for name, spec, count, wins, o, t, nseg in cases:
        note(f"wide offsets flatten {name}")
        assert t.iov_len(-1, count) == o.iov_len(-1, count), name
        for off, m in ((0, min(nseg, 4096)),) + (((nseg - 777, 1000),) if nseg > 777 else ()):
            want = max(0, min(m, nseg - off))
            hb, hl = t.iov(off, m, count)
            ob, ol = o.iov(off, m, count)
            assert np.array_equal(hb, ob) and np.array_equal(hl, ol), (name, off)
            out = torch.zeros(max(1, want) * 2, dtype=torch.int64, device="cuda")
            base = 3 << 40
            got, _ = mdt.mdt_type_iov_count_enqueue(t, count, off, out.data_ptr(), m, base, s)
            torch.cuda.synchronize()
            assert got == want == ob.size, (name, off)
            h = out.cpu().numpy()[: 2 * got].reshape(-1, 2)
            assert np.array_equal(h[:, 0] - base, ob) and np.array_equal(h[:, 1], ol), (name, off)


def test_wide_pack_windows_and_unpack(env):
    torch, mdt, host, dev, cases, opack = env
    for name, spec, count, wins, o, t, nseg in cases:
        size = t.size() * count
        full = name != "contig"
        for off, budget in ([(0, -1)] if full else []) + wins:
            note(f"wide offsets pack {name} offset={off} budget={budget}")
            exp = opack(name, o, count, off, budget)
            out = torch.full((max(1, exp.size) + 64,), 0x5A, dtype=torch.uint8, device="cuda")
            n = mdt.mdt_pack(dev.data_ptr(), count, t, off, out.data_ptr() + 3, budget)
            assert n == exp.size, (name, off, budget)
            h = out.cpu().numpy()
            assert first_diff(h[3:3 + n], exp) is None, (name, off, budget)
            assert (h[:3] == 0x5A).all() and (h[3 + n:] == 0x5A).all(), (name, off, budget)
        # unpack: the whole stream (or the window) into a zeroed buffer
        off, budget = (0, size) if full else wins[0]
        packed = opack(name, o, count, off, budget)
        exp = np.zeros(SPAN, np.uint8)
        assert o.unpack(packed, exp, 0, count, off) == packed.size
        back = torch.zeros(SPAN, dtype=torch.uint8, device="cuda")
        src = torch.from_numpy(packed).to("cuda")
        note(f"wide offsets unpack {name} offset={off} bytes={packed.size}")
        m = mdt.mdt_unpack(src.data_ptr(), packed.size, back.data_ptr(), count, t, off)
        assert m == packed.size
        torch.cuda.synchronize()
        assert _chunks_equal(torch, back, exp) is None, name
        del back, src, exp


def test_wide_offsets_in_one_batch(env):
    torch, mdt, host, dev, cases, opack = env
    s = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    plan = []
    for name, spec, count, wins, o, t, nseg in cases:
        for off, budget in wins:
            exp = opack(name, o, count, off, budget)
            plan.append((name, t, count, off, budget, exp))
    offs = np.concatenate([[0], np.cumsum([p[5].size + 8 for p in plan])])
    out = torch.zeros(int(offs[-1]), dtype=torch.uint8, device="cuda")
    b = mdt.Batch()
    for (name, t, count, off, budget, exp), o0 in zip(plan, offs):
        assert b.add_pack(dev.data_ptr(), count, t, off, out.data_ptr() + int(o0), budget) == exp.size
    # unpack requests of the non-contiguous layouts into a second buffer
    back = torch.zeros(SPAN, dtype=torch.uint8, device="cuda")
    exp_back = np.zeros(SPAN, np.uint8)
    keep = []
    for name, spec, count, wins, o, t, nseg in cases:
        if name == "contig":
            continue
        packed = opack(name, o, count, 0, -1)
        o.unpack(packed, exp_back, 0, count)
        src = torch.from_numpy(packed).to("cuda")
        keep.append(src)
        assert b.add_unpack(src.data_ptr(), packed.size, back.data_ptr(), count, t, 0) == packed.size
    for cfg in (mdt.BatchConfig(4096, 0, 0, 0, 0), mdt.BatchConfig(256, 4, 1, 1, 1), mdt.BatchConfig(1024, 0, 2, 0, 1)):
        note(f"wide offsets batch cfg={mdt.config_dict(cfg)}")
        b.set_config(cfg)
        out.zero_()
        back.zero_()
        b.launch(s)
        torch.cuda.synchronize()
        h = out.cpu().numpy()
        for (name, t, count, off, budget, exp), o0 in zip(plan, offs):
            assert first_diff(h[int(o0):int(o0) + exp.size], exp) is None, (name, off, budget)
        assert _chunks_equal(torch, back, exp_back) is None
    del b
