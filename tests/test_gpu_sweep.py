"""Parity sweeps over many seeded random nested types, every byte compared
with the oracle.

- Tiny types (every constructor, negative strides and displacements, zero
  block lengths, resized and overlapping types; tests/typegen.py), 150 per
  seed: packed at counts 1, 37 and 1000 over the whole stream and random
  byte ranges, into guard-filled outputs; flattened on the device (counts
  1 and 37); unpacked into canary-filled
  buffers when the typemap does not overlap; each seed's count-37 packs run
  as one batch in six launch configurations, and their unpacks as one batch
  in the same six and through the launch that allocates nothing.
- Medium types (counts and block lengths in the hundreds, elements spanning
  many tiles, up to 8 MiB packed), about 10 per seed: packed whole and over
  a random range, unpacked into canaries.  And typed copies between random
  pairs of types, about 15 per seed: blocking, then all of them as batch
  copies and relays (staging checked too) in four launch configurations.

MDT_SWEEP_SEEDS (default 4) sets how many seeds each sweep runs."""
import os

import numpy as np
import pytest

import bruteforce as bf
from gpu_util import first_diff, note, to_dev, to_host, zeros_dev
from oracle import OracleError
from oracle import build_type as obuild
from paper_2402_12274_amd import inputs
from typegen import buffer_for, tiny_specs

pytestmark = pytest.mark.gpu

SEEDS = int(os.environ.get("MDT_SWEEP_SEEDS", "4"))
CFGS = [(1024, 0, 2, 0, 0), (256, 4, 0, 0, 1), (4096, 2, 1, 0, 0), (1024, 0, 3, 0, 0), (512, 8, 0, 1, 1),
        (2048, 0, 2, 0, 1)]


@pytest.fixture(scope="module")
def env():
    from gpu_util import torch_cuda

    torch = torch_cuda()
    from paper_2402_12274_amd import mdt

    return torch, mdt


@pytest.mark.parametrize("seed", range(SEEDS))
def test_random_types_sweep(env, seed):
    torch, mdt = env
    ms = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    specs = tiny_specs(5000 + seed, 150)
    g = np.random.Generator(np.random.PCG64(seed))
    batch_cases = []
    for i, spec in enumerate(specs):
        note(f"sweep seed {seed} type {i}: {str(spec)[:100]}")
        tm = bf.typemap(spec)
        t = mdt.build_type(spec)
        o = obuild(spec)
        for count in (1, 37, 1000):
            size, origin = buffer_for(tm, count, pad=32)
            host = inputs.random_bytes(size, seed=seed * 1000 + i)
            src = to_dev(host)
            total = count * tm.size
            for off, mx in [(0, -1), (int(g.integers(0, total + 1)), int(g.integers(-1, total + 1))),
                            (int(g.integers(0, total + 1)), 1 + int(g.integers(0, 64)))]:
                n = max(0, total - off)
                if mx >= 0:
                    n = min(n, mx)
                out = zeros_dev(n + 48, 0xEE)
                got = mdt.mdt_pack(src.data_ptr() + origin, count, t, off, out.data_ptr() + 7, mx)
                h = to_host(out)
                exp = o.pack(host, origin, count, off, mx)
                assert got == n, (spec, count, off, mx)
                assert first_diff(h[7:7 + n], exp) is None, (spec, count, off, mx, first_diff(h[7:7 + n], exp))
                assert (h[:7] == 0xEE).all() and (h[7 + n:] == 0xEE).all(), (spec, count, "wrote outside")
            if count in (1, 37):
                # the device flatten of every segment (count form)
                nseg = o.iov_len(-1, count)[0]
                fl = torch.zeros(max(1, nseg) * 2, dtype=torch.int64, device="cuda")
                got, _ = mdt.mdt_type_iov_count_enqueue(t, count, 0, fl.data_ptr(), nseg, 1 << 40, ms)
                torch.cuda.synchronize()
                ob, ol = o.iov(0, nseg, count)
                fh = fl.cpu().numpy()[: 2 * got].reshape(-1, 2)
                assert got == nseg and np.array_equal(fh[:, 0] - (1 << 40), ob) and np.array_equal(fh[:, 1], ol), \
                    (spec, count, "flatten")
            if total > 0 and not bf.overlaps(tm, count):
                full = o.pack(host, origin, count)
                dexp = np.full(size, 0x5A, np.uint8)
                o.unpack(full, dexp, origin, count)
                dst = zeros_dev(size, 0x5A)
                fin = to_dev(full)
                mdt.mdt_unpack(fin.data_ptr(), total, dst.data_ptr() + origin, count, t, 0)
                assert first_diff(to_host(dst), dexp) is None, (spec, count, first_diff(to_host(dst), dexp))
                if count == 37:
                    batch_cases.append((t, src, origin, count, total, full, dexp, size))
    outs = [zeros_dev(c[4] + 32, 0xEE) for c in batch_cases]
    b = mdt.Batch()
    for (t, src, origin, count, total, full, _, _), out in zip(batch_cases, outs):
        b.add_pack(src.data_ptr() + origin, count, t, 0, out.data_ptr() + 5, -1)
    for cfg in CFGS:
        note(f"sweep seed {seed} batch {cfg}")
        for out in outs:
            out.fill_(0xEE)
        b.set_config(mdt.BatchConfig(*cfg))
        b.launch(ms)
        torch.cuda.synchronize()
        for k, ((t, src, origin, count, total, full, _, _), out) in enumerate(zip(batch_cases, outs)):
            h = to_host(out)
            assert first_diff(h[5:5 + total], full) is None, (cfg, k, first_diff(h[5:5 + total], full))
            assert (h[:5] == 0xEE).all() and (h[5 + total:] == 0xEE).all(), (cfg, k, "wrote outside")
    # the same requests' unpacks as one batch, into canary-filled buffers, in
    # every configuration and through the launch that allocates nothing
    ins = [to_dev(c[5]) for c in batch_cases]
    dsts = [zeros_dev(c[7], 0x5A) for c in batch_cases]
    bu = mdt.Batch()
    for (t, src, origin, count, total, full, dexp, size), fin, d in zip(batch_cases, ins, dsts):
        bu.add_unpack(fin.data_ptr(), total, d.data_ptr() + origin, count, t, 0)
    for cfg in CFGS + [None]:
        note(f"sweep seed {seed} unpack batch {cfg}")
        for d in dsts:
            d.fill_(0x5A)
        if cfg is None:
            bu.set_config(mdt.BatchConfig(1024, 0, 2, 0, 1))
            bu.launch_noalloc(ms)
        else:
            bu.set_config(mdt.BatchConfig(*cfg))
            bu.launch(ms)
        torch.cuda.synchronize()
        for k, (c, d) in enumerate(zip(batch_cases, dsts)):
            assert first_diff(to_host(d), c[6]) is None, (cfg, k, first_diff(to_host(d), c[6]))


BASICS = ["BYTE", "INT16", "INT32", "FLOAT", "DOUBLE", "INT64"]


def _medium(g, depth=0):
    """A random type with counts and block lengths in the hundreds."""
    if depth >= 3 or g.random() < 0.2 + 0.2 * depth:
        return ("basic", BASICS[int(g.integers(0, len(BASICS)))])
    c = _medium(g, depth + 1)
    k = int(g.integers(0, 8))
    r = lambda lo, hi: int(g.integers(lo, hi + 1))  # noqa: E731
    if k == 0:
        return ("contiguous", r(1, 300), c)
    if k == 1:
        return ("vector", r(1, 300), r(1, 20), r(-30, 40), c)
    if k == 2:
        return ("hvector", r(1, 200), r(1, 10), r(-500, 3000), c)
    if k == 3:
        n = r(1, 400)
        disps = [r(-5000, 50000) for _ in range(n)]
        return ("hindexed", [r(0, 12) for _ in range(n)], sorted(disps) if g.random() < 0.5 else disps, c)
    if k == 4:
        n = r(1, 4)
        kids = [c] + [_medium(g, depth + 1) for _ in range(n - 1)]
        return ("struct", [r(0, 30) for _ in range(n)], sorted(r(-64, 4096) for _ in range(n)), kids)
    if k == 5:
        nd = r(1, 3)
        sizes = [r(1, 40) for _ in range(nd)]
        subs = [r(1, s) for s in sizes]
        starts = [r(0, s - u) for s, u in zip(sizes, subs)]
        return ("subarray", sizes, subs, starts, "C" if g.random() < 0.6 else "F", c)
    if k == 6:
        return ("resized", r(-64, 64), r(1, 4096), c)
    return ("indexed_block", r(1, 8), [r(-100, 2000) for _ in range(r(1, 200))], c)


def _span(a, count):
    """(bytes, origin) of a buffer covering (count x type), 32 guard bytes a side."""
    ext = a["extent"]
    lo = min(a["true_lb"], a["true_lb"] + (count - 1) * ext)
    hi = max(a["true_lb"] + a["true_extent"], a["true_lb"] + a["true_extent"] + (count - 1) * ext)
    return hi - lo + 64, 32 - lo


@pytest.mark.parametrize("seed", range(SEEDS))
def test_medium_types_and_copies_sweep(env, seed):
    torch, mdt = env
    ms = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    g = np.random.Generator(np.random.PCG64(9000 + seed))
    for i in range(12):
        spec = _medium(g)
        o = obuild(spec)
        a = o.attrs()
        if a["size"] == 0 or a["size"] > (8 << 20) or a["true_extent"] > (256 << 20) or abs(a["extent"]) > (64 << 20):
            continue
        count = int(g.integers(1, 4))
        size, origin = _span(a, count)
        if size > (512 << 20):
            continue
        note(f"sweep seed {seed} medium {i}: {str(spec)[:100]}")
        t = mdt.build_type(spec)
        host = inputs.random_bytes(size, seed=seed * 100 + i)
        src = to_dev(host)
        total = count * a["size"]
        for off, mx in [(0, -1), (int(g.integers(0, total)), int(g.integers(1, total + 1)))]:
            n = max(0, total - off) if mx < 0 else min(mx, max(0, total - off))
            out = zeros_dev(n + 48, 0xEE)
            got = mdt.mdt_pack(src.data_ptr() + origin, count, t, off, out.data_ptr() + 3, mx)
            h = to_host(out)
            exp = o.pack(host, origin, count, off, mx)
            assert got == n and first_diff(h[3:3 + n], exp) is None, (spec, count, off, mx)
            assert (h[:3] == 0xEE).all() and (h[3 + n:] == 0xEE).all(), (spec, "wrote outside")
        full = o.pack(host, origin, count)
        dexp = np.full(size, 0x5A, np.uint8)
        try:
            o.unpack(full, dexp, origin, count)
        except OracleError:
            continue  # overlapping typemap: unpack is rejected (checked elsewhere)
        dst = zeros_dev(size, 0x5A)
        fin = to_dev(full)
        mdt.mdt_unpack(fin.data_ptr(), total, dst.data_ptr() + origin, count, t, 0)
        assert first_diff(to_host(dst), dexp) is None, (spec, count, first_diff(to_host(dst), dexp))
    # typed copies and relays between random pairs of tiny types
    specs = tiny_specs(7000 + seed, 60, allow_overlap=False)
    cases = []
    for j in range(0, len(specs) - 1, 2):
        sa, sb = specs[j], specs[j + 1]
        za, zb = bf.typemap(sa).size, bf.typemap(sb).size
        if za == 0 or zb == 0:
            continue
        ca = int(g.integers(1, 40))
        cb = -(-ca * za // zb) + int(g.integers(0, 3))
        if bf.overlaps(bf.typemap(sb), cb):
            continue
        note(f"sweep seed {seed} copy {j}: {str(sa)[:50]} x{ca} -> {str(sb)[:50]} x{cb}")
        ta, tb = mdt.build_type(sa), mdt.build_type(sb)
        ns, org_s = buffer_for(bf.typemap(sa), ca, pad=19)
        nd, org_d = buffer_for(bf.typemap(sb), cb, pad=23)
        src_host = inputs.random_bytes(ns, seed=seed * 1000 + j)
        total = ca * za
        off, mx = int(g.integers(0, total)), int(g.integers(-1, total + 1))
        packed = obuild(sa).pack(src_host, org_s, ca, off, mx)
        dst_host = np.full(nd, 0xA5, np.uint8)
        exp = dst_host.copy()
        if packed.size:
            obuild(sb).unpack(packed, exp, org_d, cb, off)
        src = to_dev(src_host)
        dst = to_dev(dst_host)
        got = mdt.mdt_typed_copy(src.data_ptr() + org_s, ca, ta, dst.data_ptr() + org_d, cb, tb, off, mx)
        assert got == packed.size and first_diff(to_host(dst), exp) is None, (sa, sb, off, mx)
        cases.append((ta, tb, src, org_s, ca, org_d, cb, off, mx, packed, exp, dst_host))
    for cfg in [(1024, 0, 2, 0, 0), (256, 4, 0, 0, 1), (4096, 2, 1, 0, 0), (1024, 0, 3, 0, 0)]:
        note(f"sweep seed {seed} copies and relays, batch {cfg}")
        b = mdt.Batch()
        dsts, stg = [], []
        for k, (ta, tb, src, org_s, ca, org_d, cb, off, mx, packed, exp, dst_host) in enumerate(cases):
            d = to_dev(dst_host)
            dsts.append(d)
            if k % 2:
                b.add_copy(src.data_ptr() + org_s, ca, ta, d.data_ptr() + org_d, cb, tb, off, mx)
                stg.append(None)
            else:
                st = zeros_dev(packed.size + 16, 0)
                stg.append(st)
                b.add_relay(src.data_ptr() + org_s, ca, ta, st.data_ptr() + 5, d.data_ptr() + org_d, cb, tb, off, mx)
        b.set_config(mdt.BatchConfig(*cfg))
        b.launch(ms)
        torch.cuda.synchronize()
        for k, c in enumerate(cases):
            assert first_diff(to_host(dsts[k]), c[10]) is None, (cfg, k, "destination")
            if stg[k] is not None:
                assert first_diff(to_host(stg[k])[5:5 + c[9].size], c[9]) is None, (cfg, k, "staging")
