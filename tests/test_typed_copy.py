"""Typed copy (layout to layout, no staging buffer) against the oracle.

The copy of stream bytes [off, off + n) from (ca x A) to (cb x B) must equal
the oracle's pack of that range from A followed by its unpack into B at the
same stream positions, byte for byte, with every byte of the destination
outside B's typemap left as it was (canary-filled buffers).  Host checks run
without a GPU: truncation, overlapping destinations and bad arguments are
rejected before any device work.
"""
import ctypes

import numpy as np
import pytest

import bruteforce as bf
from oracle import build_type as obuild
from paper_2402_12274_amd import inputs
from typegen import buffer_for, tiny_specs

mdt = pytest.importorskip("paper_2402_12274_amd.mdt")

D = inputs.DOUBLE


def test_copy_errors_on_host():
    a = mdt.build_type(("contiguous", 10, D))
    b = mdt.build_type(("contiguous", 8, D))
    over = mdt.build_type(("hvector", 2, 2, 8, D))  # covers bytes 8..15 twice
    n = ctypes.c_int64(-7)
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every call below fails before device work
    # 80 source bytes into a 64-byte destination stream
    assert mdt._lib.mdt_typed_copy(fake, 1, a.h, fake, 1, b.h, 0, -1, ctypes.byref(n)) == mdt.ERR_TRUNCATE
    # ... also when the offset leaves too little room (64 bytes from 16 of 64)
    assert mdt._lib.mdt_typed_copy(fake, 1, a.h, fake, 1, b.h, 16, 64, ctypes.byref(n)) == mdt.ERR_TRUNCATE
    # overlapping destination typemap
    assert mdt._lib.mdt_typed_copy(fake, 1, b.h, fake, 2, over.h, 0, 16, ctypes.byref(n)) == mdt.ERR_OVERLAP
    # bad arguments
    assert mdt._lib.mdt_typed_copy(fake, 1, b.h, fake, 1, b.h, -1, -1, ctypes.byref(n)) == mdt.ERR_ARG
    assert mdt._lib.mdt_typed_copy(fake, 1, b.h, fake, 1, b.h, 0, -2, ctypes.byref(n)) == mdt.ERR_ARG
    assert mdt._lib.mdt_typed_copy(fake, 1, b.h, fake, 1, b.h, 0, -1, None) == mdt.ERR_ARG
    assert mdt._lib.mdt_typed_copy(None, 1, b.h, fake, 1, b.h, 0, -1, ctypes.byref(n)) == mdt.ERR_ARG
    # the blocking pack and unpack reject a NULL byte-count output as well
    assert mdt._lib.mdt_pack(fake, 1, b.h, 0, fake, -1, None) == mdt.ERR_ARG
    assert mdt._lib.mdt_unpack(fake, 8, fake, 1, b.h, 0, None) == mdt.ERR_ARG
    assert n.value == -7  # outputs untouched on error


def _expected(src_host, sa, ca, org_s, dst_host, sb, cb, org_d, off, mx):
    oa, ob = obuild(sa), obuild(sb)
    packed = oa.pack(src_host, org_s, ca, off, mx)
    exp = dst_host.copy()
    ob.unpack(packed, exp, org_d, cb, off)
    return exp, packed.size


def _pairs(seed, n):
    """(A, ca, B, cb) with size(B)*cb >= size(A)*ca and B free of overlap."""
    g = np.random.Generator(np.random.PCG64(seed))
    specs = tiny_specs(seed, 3 * n, allow_overlap=False)
    out = []
    i = 0
    while len(out) < n and i + 1 < len(specs):
        sa, sb = specs[i], specs[i + 1]
        i += 2
        za, zb = bf.typemap(sa).size, bf.typemap(sb).size
        if za == 0 or zb == 0:
            continue
        ca = int(g.integers(1, 4))
        cb = -(-ca * za // zb) + int(g.integers(0, 2))
        if bf.overlaps(bf.typemap(sb), cb):
            continue
        out.append((sa, ca, sb, cb))
    return out


PAIRS = _pairs(77, 40)


@pytest.mark.gpu
@pytest.mark.parametrize("i", range(len(PAIRS)))
def test_copy_random_pairs(i):
    from gpu_util import first_diff, note, to_dev, to_host, torch_cuda

    torch_cuda()
    sa, ca, sb, cb = PAIRS[i]
    note(f"typed copy pair {i}: {str(sa)[:50]} x{ca} -> {str(sb)[:50]} x{cb}")
    ta, tb = mdt.build_type(sa), mdt.build_type(sb)
    ns, org_s = buffer_for(bf.typemap(sa), ca, pad=19)
    nd, org_d = buffer_for(bf.typemap(sb), cb, pad=23)
    src_host = inputs.random_bytes(ns, seed=300 + i)
    src = to_dev(src_host)
    total = ca * bf.typemap(sa).size
    for off, mx in [(0, -1), (3, 17), (total // 2, -1), (1, total)]:
        dst_host = np.full(nd, 0xA5, np.uint8)
        exp, n = _expected(src_host, sa, ca, org_s, dst_host, sb, cb, org_d, off, mx)
        dst = to_dev(dst_host)
        got = mdt.mdt_typed_copy(src.data_ptr() + org_s, ca, ta, dst.data_ptr() + org_d, cb, tb, off, mx)
        assert got == n
        assert first_diff(to_host(dst), exp) is None, (sa, sb, off, mx)


@pytest.mark.gpu
def test_copy_workload_layouts():
    # periodic halo self-exchange (interior face -> opposite ghost face of
    # the same array), records <-> contiguous, irregular -> strided, with
    # chunked ranges that cross tiles and end ragged
    from gpu_util import first_diff, note, to_dev, to_host, torch_cuda

    torch_cuda()
    n = 96
    host = inputs.random_bytes(n ** 3 * 8, seed=41)
    for w in (1, 4):
        for dim in (0, 1, 2):
            src_spec = inputs.halo_face(n, w, dim, "lo")
            sub = [n - 2 * w] * 3
            st = [w] * 3
            sub[dim] = w
            st[dim] = n - w  # ghost layer on the far side
            dst_spec = ("subarray", [n, n, n], sub, st, "C", D)
            note(f"halo self-exchange w={w} dim={dim}")
            ta, tb = mdt.build_type(src_spec), mdt.build_type(dst_spec)
            exp, nb = _expected(host, src_spec, 1, 0, host, dst_spec, 1, 0, 0, -1)
            arr = to_dev(host)
            got = mdt.mdt_typed_copy(arr.data_ptr(), 1, ta, arr.data_ptr(), 1, tb, 0, -1)
            assert got == nb
            assert first_diff(to_host(arr), exp) is None, (w, dim)
    # particle records to a contiguous array and back, in 64 KiB - 1 pieces
    cnt = 30001
    rec = inputs.particle_struct()
    flat = ("contiguous", 33 * cnt, inputs.BYTE)
    src_host = inputs.random_bytes(cnt * 40, seed=42)
    for sa, ca, sb, cb, nsrc, ndst in [(rec, cnt, flat, 1, cnt * 40, 33 * cnt), (flat, 1, rec, cnt, 33 * cnt, cnt * 40)]:
        note(f"records copy {sa[0]} -> {sb[0]}")
        ta, tb = mdt.build_type(sa), mdt.build_type(sb)
        sh = src_host[:nsrc]
        src = to_dev(sh)
        dst_host = np.full(ndst, 0x3C, np.uint8)
        dst = to_dev(dst_host)
        exp, total = _expected(sh, sa, ca, 0, dst_host, sb, cb, 0, 0, -1)
        off = 0
        while off < total:
            off += mdt.mdt_typed_copy(src.data_ptr(), ca, ta, dst.data_ptr(), cb, tb, off, (1 << 16) - 1)
        assert first_diff(to_host(dst), exp) is None
    # irregular blocks into a strided vector of bytes
    lens, disps = inputs.hindexed_blocks(nblocks=20000, span=1 << 21, seed=43)
    sa = inputs.hindexed_type(lens, disps)
    size = int(np.asarray(lens).sum())
    sb = ("vector", size, 1, 3, inputs.BYTE)
    note("hindexed -> vector")
    ta, tb = mdt.build_type(sa), mdt.build_type(sb)
    sh = inputs.random_bytes(1 << 21, seed=44)
    dst_host = np.full(3 * size, 0x11, np.uint8)
    exp, total = _expected(sh, sa, 1, 0, dst_host, sb, 1, 0, 0, -1)
    src, dst = to_dev(sh), to_dev(dst_host)
    assert mdt.mdt_typed_copy(src.data_ptr(), 1, ta, dst.data_ptr(), 1, tb, 0, -1) == total
    assert first_diff(to_host(dst), exp) is None


@pytest.mark.gpu
def test_copy_enqueue_stream_order():
    # a copy enqueued between two packs on one stream sees the first pack's
    # output and is seen by the second
    from gpu_util import first_diff, to_dev, to_host, torch_cuda

    torch = torch_cuda()
    t = mdt.build_type(("vector", 4096, 1, 2, D))
    flat = mdt.build_type(("contiguous", 4096, D))
    host = inputs.random_bytes(4096 * 16, seed=45)
    src = to_dev(host)
    mid = torch.zeros(4096 * 8, dtype=torch.uint8, device="cuda")
    back = torch.zeros(4096 * 16, dtype=torch.uint8, device="cuda")
    out = torch.zeros(4096 * 8, dtype=torch.uint8, device="cuda")
    ms = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    mdt.mdt_pack_enqueue(src.data_ptr(), 1, t, 0, mid.data_ptr(), -1, ms)
    n, req = mdt.mdt_typed_copy_enqueue(mid.data_ptr(), 1, flat, back.data_ptr(), 1, t, 0, -1, ms, want_request=True)
    mdt.mdt_pack_enqueue(back.data_ptr(), 1, t, 0, out.data_ptr(), -1, ms)
    req.wait()
    torch.cuda.synchronize()
    exp = host.reshape(4096, 16)[:, :8].reshape(-1)
    assert n == 4096 * 8
    assert first_diff(to_host(out), exp) is None


@pytest.mark.gpu
def test_copy_requests_in_a_batch():
    # the six halo self-exchange copies of one width as batch requests, next
    # to pack and unpack requests of other buffers; every result equals the
    # oracle's, for request and address order
    from gpu_util import first_diff, note, to_dev, to_host, torch_cuda

    torch = torch_cuda()
    n, w = 96, 2
    host = inputs.random_bytes(n ** 3 * 8, seed=51)
    exp = host.copy()
    copies = []
    for dim in (0, 1, 2):
        for side in ("lo", "hi"):
            src_spec = inputs.halo_face(n, w, dim, side)
            sub = [n - 2 * w] * 3
            st = [w] * 3
            sub[dim] = w
            st[dim] = n - w if side == "lo" else 0
            dst_spec = ("subarray", [n, n, n], sub, st, "C", D)
            copies.append((src_spec, dst_spec))
            packed = obuild(src_spec).pack(host, 0, 1)
            obuild(dst_spec).unpack(packed, exp, 0, 1)
    rec = inputs.particle_struct()
    rh = inputs.random_bytes(5000 * 40, seed=52)
    rexp_pack = obuild(rec).pack(rh, 0, 5000)
    ms = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    for wgs, order, pol in ((0, 0, 0), (4, 1, 0), (0, 0, 2), (0, 0, 3)):
        note(f"batch with copies wgs={wgs} order={order} policy={pol}")
        arr = to_dev(host)
        rsrc = to_dev(rh)
        rout = torch.zeros(rexp_pack.size, dtype=torch.uint8, device="cuda")
        rback = torch.zeros(5000 * 40, dtype=torch.uint8, device="cuda")
        b = mdt.Batch()
        tr = mdt.build_type(rec)
        b.add_pack(rsrc.data_ptr(), 5000, tr, 0, rout.data_ptr(), -1)
        for sa, sb in copies:
            b.add_copy(arr.data_ptr(), 1, mdt.build_type(sa), arr.data_ptr(), 1, mdt.build_type(sb), 0, -1)
        pk = to_dev(rexp_pack)
        b.add_unpack(pk.data_ptr(), rexp_pack.size, rback.data_ptr(), 5000, tr, 0)
        b.set_config(mdt.BatchConfig(1024, wgs, pol, 1, order))
        b.launch(ms)
        torch.cuda.synchronize()
        assert first_diff(to_host(arr), exp) is None
        assert first_diff(to_host(rout), rexp_pack) is None
        rexp_back = np.zeros(5000 * 40, np.uint8)
        obuild(rec).unpack(rexp_pack, rexp_back, 0, 5000)
        assert first_diff(to_host(rback), rexp_back) is None
