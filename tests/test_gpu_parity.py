"""GPU parity: every byte the gfx950 kernels move must equal the oracle's.

Pack, partial pack, unpack (into canary-filled buffers, so gaps are proven
untouched) and the device flatten are compared element by element with the
oracle on the same seeded inputs: random tiny types of every constructor at
odd buffer alignments, the small vector case, and mid-size versions of the
halo-face, hindexed and particle-record layouts that span many tiles and
end in a ragged tail.  Full-size workloads are in test_gpu_fullsize.py.
"""
import numpy as np
import pytest

import bruteforce as bf
from gpu_util import first_diff, note, to_dev, to_host, zeros_dev
from oracle import build_type as obuild
from paper_2402_12274_amd import inputs
from typegen import buffer_for, tiny_specs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdt():
    from gpu_util import torch_cuda

    torch_cuda()
    from paper_2402_12274_amd import mdt as m

    return m


def _pack_dev(mdt, t, src_dev, origin, count, off, mx, out_shift=0):
    total = count * t.size()
    n = max(0, total - off)
    if mx >= 0:
        n = min(n, mx)
    out = zeros_dev(n + 32, 0xEE)
    got = mdt.mdt_pack(src_dev.data_ptr() + origin, count, t, off, out.data_ptr() + out_shift, mx)
    assert got == n
    h = to_host(out)
    assert (h[:out_shift] == 0xEE).all() and (h[out_shift + n:] == 0xEE).all(), "pack wrote outside its output"
    return h[out_shift:out_shift + n]


SPECS = tiny_specs(99, 120) + [
    # one run at a nonzero offset inside the element, alone and repeated
    ("hindexed", [1, 1], [-19, -15], ("basic", "INT32")),
    ("contiguous", 2, ("hindexed", [1, 1], [-19, -15], ("basic", "INT32"))),
    ("contiguous", 3, ("hindexed", [1, 1, 1], [5, 9, 13], ("basic", "INT32"))),
]


@pytest.mark.parametrize("i", range(len(SPECS)))
def test_random_types_pack_unpack(mdt, i):
    spec = SPECS[i]
    note(f"random type {i}: {spec}")
    tm = bf.typemap(spec)
    t = mdt.build_type(spec)
    o = obuild(spec)
    for count in (1, 3):
        size, origin = buffer_for(tm, count, pad=64)
        host = inputs.random_bytes(size, seed=1000 + i)
        src = to_dev(host)
        total = count * tm.size
        full = o.pack(host, origin, count)
        for shift in (0, 3, 8):
            got = _pack_dev(mdt, t, src, origin, count, 0, -1, shift)
            assert first_diff(got, full) is None, (spec, count, shift, first_diff(got, full))
        for off, mx in [(1, 5), (total // 2, 17), (3, total), (total, 4), (total + 2, -1), (0, 0)]:
            got = _pack_dev(mdt, t, src, origin, count, off, mx, 5)
            exp = o.pack(host, origin, count, off, mx)
            assert first_diff(got, exp) is None, (spec, count, off, mx)
        if bf.overlaps(tm, count):
            dst = zeros_dev(size, 0x5A)
            with pytest.raises(mdt.MdtError) as e:
                mdt.mdt_unpack(to_dev(full).data_ptr(), total, dst.data_ptr() + origin, count, t, 0)
            assert e.value.code == mdt.ERR_OVERLAP
            continue
        for off, n in [(0, total), (total // 3, total - total // 3), (1, max(0, min(7, total - 1)))]:
            canary = np.full(size, 0x5A, np.uint8)
            exp = canary.copy()
            if n > 0:
                o.unpack(full[off:off + n], exp, origin, count, off)
            dst = to_dev(canary)
            packed = zeros_dev(n + 16, 0)
            packed[3:3 + n] = to_dev(full[off:off + n]) if n > 0 else packed[3:3]
            got = mdt.mdt_unpack(packed.data_ptr() + 3, n, dst.data_ptr() + origin, count, t, off)
            assert got == n
            h = to_host(dst)
            assert first_diff(h, exp) is None, (spec, count, off, n, first_diff(h, exp))


def test_small_vector_case(mdt):
    note("small vector case")
    spec = inputs.vector_small()
    t = mdt.build_type(spec)
    o = obuild(spec)
    assert t.iov_len(-1) == o.iov_len(-1) == (1024, 8192)
    assert t.iov_len(4096) == o.iov_len(4096) == (512, 4096)
    b, ln = t.iov(512, 4)
    ob, ol = o.iov(512, 4)
    assert np.array_equal(b, ob) and np.array_equal(ln, ol) and b[0] == 8192
    host = inputs.random_bytes(16384, seed=inputs.DEFAULT_SEED)
    src = to_dev(host)
    packed = _pack_dev(mdt, t, src, 0, 1, 0, -1)
    assert first_diff(packed, o.pack(host, 0, 1)) is None
    dst = zeros_dev(16384, 0)
    mdt.mdt_unpack(to_dev(packed).data_ptr(), 8192, dst.data_ptr(), 1, t, 0)
    h = to_host(dst)
    exp = np.zeros(16384, np.uint8)
    o.unpack(packed, exp, 0, 1)
    assert first_diff(h, exp) is None
    # round trip: covered bytes restored, the gaps stay zero
    view = host.reshape(1024, 16)
    assert np.array_equal(h.reshape(1024, 16)[:, :8], view[:, :8]) and not h.reshape(1024, 16)[:, 8:].any()


def _layout_case(mdt, spec, count, src_bytes, origin, seed, chunk):
    t = mdt.build_type(spec)
    o = obuild(spec)
    host = inputs.random_bytes(src_bytes, seed=seed)
    src = to_dev(host)
    full = o.pack(host, origin, count)
    got = _pack_dev(mdt, t, src, origin, count, 0, -1)
    assert first_diff(got, full) is None, first_diff(got, full)
    # partial packs with a byte budget concatenate to the full stream
    parts = []
    off = 0
    while off < full.size:
        parts.append(_pack_dev(mdt, t, src, origin, count, off, chunk, off % 13))
        off += chunk
    assert first_diff(np.concatenate(parts), full) is None
    # unpack into a canary buffer, chunk by chunk
    canary = np.full(src_bytes, 0x77, np.uint8)
    exp = canary.copy()
    o.unpack(full, exp, origin, count)
    dst = to_dev(canary)
    pk = to_dev(full)
    off = 0
    while off < full.size:
        n = min(chunk, full.size - off)
        mdt.mdt_unpack(pk.data_ptr() + off, n, dst.data_ptr() + origin, count, t, off)
        off += n
    h = to_host(dst)
    assert first_diff(h, exp) is None, first_diff(h, exp)


def test_halo_faces_midsize(mdt):
    n = 96
    for label, spec in inputs.halo_faces(n):
        note(f"halo face {label} n={n}")
        _layout_case(mdt, spec, 1, n ** 3 * 8, 0, seed=hash(label) & 0xffff, chunk=(1 << 14) + 9)


def test_hindexed_midsize(mdt):
    lens, disps = inputs.hindexed_blocks(nblocks=20000, span=1 << 22, seed=3)
    note("hindexed midsize")
    _layout_case(mdt, inputs.hindexed_type(lens, disps), 1, 1 << 22, 0, seed=4, chunk=(1 << 16) + 3)
    lens, disps = inputs.hindexed_blocks(nblocks=20000, span=1 << 22, seed=5, permute=False)
    _layout_case(mdt, inputs.hindexed_type(lens, disps), 2, 1 << 23, 0, seed=6, chunk=1 << 16)


def test_particle_records_midsize(mdt):
    note("particle records midsize")
    count = 50001
    _layout_case(mdt, inputs.particle_struct(), count, count * 40, 0, seed=8, chunk=(1 << 16) - 1)


def test_long_runs_partial(mdt):
    # runs longer than a tile (whole tiles inside one run) with ragged edges:
    # odd byte strides, misaligned output pointers, budgets off the 16-B grid
    cases = [
        (("subarray", [64, 4096], [40, 3001], [7, 13], "C", inputs.DOUBLE), 1, 64 * 4096 * 8, 0, (1 << 17) + 5),
        (("hvector", 9, 20011, 20011 + 4099, inputs.BYTE), 2, 2 * 9 * 24110 + 64, 3, 40009),
        (("vector", 5, 4100, 4100 + 3, ("basic", "FLOAT")), 3, 3 * 5 * 4103 * 4, 1, 1 << 16),
    ]
    for spec, count, nbytes, origin, chunk in cases:
        note(f"long runs {spec[0]} count={count}")
        _layout_case(mdt, spec, count, nbytes, origin, seed=count * 7 + 1, chunk=chunk)


C, I16, I32, U8 = ("basic", "CHAR"), ("basic", "INT16"), ("basic", "INT32"), ("basic", "UINT8")
RECORD_CASES = [
    # (spec, count, origin, chunk, (records, pack_table, unpack_table)):
    # record views with odd strides, gaps at both ends of a record, map order
    # unlike address order, records of many small runs large enough for the
    # byte-table paths (U > 256, X > 1024), interleaved records (unpack on the
    # chunk path), and records of one long run (left to the chunk path)
    (("resized", 0, 9, ("struct", [1, 1, 1], [0, 2, 7], [C, I16, C])), 30001, 3, 4099, (1, 2, 2)),
    (("hvector", 20000, 3, 4, U8), 1, 1, 5003, (1, 2, 2)),
    (("hvector", 5000, 1, 12, I32), 1, 2, 1 << 12, (1, 2, 2)),
    (("struct", [1, 1, 3], [16, 0, 8], [inputs.DOUBLE, I32, C]), 40000, 5, 65537, (1, 2, 2)),
    (("resized", 0, 600, ("hindexed", [8] * 40, [14 * i + i % 3 for i in range(40)], C)), 3000, 0, (1 << 15) + 1,
     (1, 1, 2)),
    (("resized", 0, 1200, ("hindexed", [5] * 60, [19 * i + i % 2 for i in range(60)], C)), 500, 7, 30011, (1, 1, 1)),
    (("resized", 0, 320, ("contiguous", 75, I32)), 3000, 0, (1 << 15) + 1, (0, 0, 0)),
    (("resized", 0, 8, ("struct", [1, 1], [0, 12], [I32, I32])), 20000, 1, 9999, (1, 2, 0)),
]


@pytest.mark.parametrize("i", range(len(RECORD_CASES)))
def test_record_layouts(mdt, i):
    spec, count, origin, chunk, path = RECORD_CASES[i]
    note(f"record layout {i}: {str(spec)[:70]} count={count}")
    info = mdt.build_type(spec).layout_info()
    assert (info["records"], info["pack_table"], info["unpack_table"]) == path, info
    o = obuild(spec)
    a = o.attrs()
    nbytes = origin + (count - 1) * a["extent"] + a["true_ub"] + 16
    _layout_case(mdt, spec, count, nbytes, origin, seed=100 + i, chunk=chunk)


def test_record_split_unpack_in_one_batch(mdt):
    # two halves of one stream unpacked into one buffer by one launch: the
    # dword that straddles the split is assembled by both requests, each
    # writing only the bytes of its own half
    from gpu_util import torch_cuda

    torch = torch_cuda()
    spec = ("resized", 0, 9, ("struct", [1, 1, 1], [0, 2, 7], [C, I16, C]))
    count = 20000
    t = mdt.build_type(spec)
    o = obuild(spec)
    host = inputs.random_bytes(count * 9 + 16, seed=31)
    full = o.pack(host, 0, count)
    pk = to_dev(full)
    ms = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    for split in (full.size // 2, 12345, 4 * 9 * 1000 + 1):
        canary = np.full(host.size, 0x5A, np.uint8)
        exp = canary.copy()
        o.unpack(full, exp, 0, count)
        dst = to_dev(canary)
        b = mdt.Batch()
        b.add_unpack(pk.data_ptr(), split, dst.data_ptr(), count, t, 0)
        b.add_unpack(pk.data_ptr() + split, full.size - split, dst.data_ptr(), count, t, split)
        b.launch(ms)
        torch.cuda.synchronize()
        assert first_diff(to_host(dst), exp) is None, split


def test_contiguous_and_degenerate(mdt):
    note("contiguous / degenerate")
    host = inputs.random_bytes(1 << 20, seed=9)
    src = to_dev(host)
    t = mdt.build_type(("contiguous", 1 << 17, inputs.DOUBLE))
    for off, mx, shift in [(0, -1, 0), (5, 99999, 7), (1 << 19, 1 << 18, 1)]:
        got = _pack_dev(mdt, t, src, 0, 1, off, mx, shift)
        exp = host[off:off + (len(host) - off if mx < 0 else mx)]
        assert first_diff(got, exp) is None
    # count 0, offset past the end, zero budget: no bytes, no writes
    for cnt, off, mx in [(0, 0, -1), (1, 1 << 20, -1), (1, 100, 0)]:
        assert _pack_dev(mdt, t, src, 0, cnt, off, mx).size == 0
    # an empty type
    e = mdt.build_type(("vector", 0, 1, 2, inputs.DOUBLE))
    assert _pack_dev(mdt, e, src, 0, 5, 0, -1).size == 0
    # regressions: empty types whose parts are not representable commit, and
    # an unpack of 2^40 elements of an empty type returns at once
    huge = ("resized", -(1 << 61), 1 << 62, inputs.DOUBLE)
    e2 = mdt.build_type(("hvector", 0, 3, 1 << 20, huge))
    assert _pack_dev(mdt, e2, src, 0, 1, 0, -1).size == 0
    e3 = mdt.build_type(("resized", 0, 8, ("vector", 0, 1, 2, inputs.DOUBLE)))
    assert mdt.mdt_unpack(src.data_ptr(), 0, src.data_ptr(), 1 << 40, e3, 0) == 0
    # truncation is an error and writes nothing
    dst = zeros_dev(64, 0)
    with pytest.raises(mdt.MdtError) as ex:
        mdt.mdt_unpack(src.data_ptr(), 65, dst.data_ptr(), 1, mdt.build_type(("contiguous", 8, inputs.DOUBLE)), 0)
    assert ex.value.code == mdt.ERR_TRUNCATE
    assert not to_host(dst).any()


def test_device_flatten_matches_oracle(mdt):
    import ctypes

    torch = pytest.importorskip("torch")
    specs = [inputs.vector_small(), inputs.particle_struct(), inputs.halo_face(64, 1, 2, "lo"),
             inputs.halo_face(64, 4, 1, "hi"), ("contiguous", 4, ("vector", 3, 1, 2, inputs.DOUBLE))]
    lens, disps = inputs.hindexed_blocks(nblocks=5000, span=1 << 20, seed=11)
    specs.append(inputs.hindexed_type(lens, disps))
    specs += tiny_specs(5, 30)
    # one run at a nonzero offset, alone and repeated (regression)
    I32 = ("basic", "INT32")
    specs += [("hindexed", [1, 1], [-19, -15], I32), ("contiguous", 2, ("hindexed", [1, 1], [-19, -15], I32)),
              ("contiguous", 3, ("hindexed", [1, 1, 1], [5, 9, 13], I32))]
    s = mdt.Stream(0)
    for spec in specs:
        note(f"flatten {str(spec)[:80]}")
        t = mdt.build_type(spec)
        o = obuild(spec)
        nseg = o.iov_len(-1)[0]
        for off, m in [(0, nseg), (nseg // 3, 1000), (nseg, 5)]:
            out = torch.zeros(max(1, min(m, max(0, nseg - off))) * 2, dtype=torch.int64, device="cuda")
            base = 1 << 40
            got, _ = mdt.mdt_type_iov_enqueue(t, off, out.data_ptr(), m, base, s)
            torch.cuda.synchronize()
            ob, ol = o.iov(off, m)
            assert got == ob.size
            h = out.cpu().numpy()[: 2 * got].reshape(-1, 2)
            assert np.array_equal(h[:, 0] - base, ob) and np.array_equal(h[:, 1], ol), spec
    assert ctypes.sizeof(mdt.Iov) == 16


def test_device_flatten_count_matches_oracle(mdt):
    # the count form on the device: element segments repeated at multiples
    # of the extent, merged across element boundaries where they touch
    torch = pytest.importorskip("torch")
    specs = [inputs.vector_small(), inputs.particle_struct(), inputs.halo_face(64, 1, 2, "lo"),
             ("resized", 0, 12, ("vector", 2, 1, 2, ("basic", "INT32"))), ("resized", 0, 24, ("contiguous", 3, inputs.DOUBLE)),
             ("contiguous", 4, ("vector", 3, 1, 2, inputs.DOUBLE))]
    lens, disps = inputs.hindexed_blocks(nblocks=3000, span=1 << 20, seed=12)
    specs.append(inputs.hindexed_type(lens, disps))
    specs += tiny_specs(6, 20)
    s = mdt.Stream(0)
    for spec in specs:
        t = mdt.build_type(spec)
        o = obuild(spec)
        for count in (0, 2, 5):
            note(f"flatten count={count} {str(spec)[:70]}")
            nseg = o.iov_len(-1, count)[0]
            for off, m in [(0, nseg), (nseg // 3, 777), (max(nseg - 2, 0), 5), (nseg, 5)]:
                want = max(0, min(m, nseg - off))
                out = torch.zeros(max(1, want) * 2, dtype=torch.int64, device="cuda")
                base = 1 << 40
                got, _ = mdt.mdt_type_iov_count_enqueue(t, count, off, out.data_ptr(), m, base, s)
                torch.cuda.synchronize()
                ob, ol = o.iov(off, m, count)
                assert got == ob.size == want
                h = out.cpu().numpy()[: 2 * got].reshape(-1, 2)
                assert np.array_equal(h[:, 0] - base, ob) and np.array_equal(h[:, 1], ol), (spec, count, off)


def test_darray_random_small(mdt):
    """Random distributed arrays (every distribution, both orders, gapped
    element types): full and partial packs at odd output alignments and
    unpack into canaries, against the oracle."""
    from typegen import darray_specs

    for i, spec in enumerate(darray_specs(123, 60)):
        note(f"darray small {i}: {spec}")
        t = mdt.build_type(spec)
        o = obuild(spec)
        a = o.attrs()
        if a["size"] == 0:
            continue
        size = a["extent"] + 64
        host = inputs.random_bytes(size, seed=500 + i)
        src = to_dev(host)
        full = o.pack(host, 32, 1)
        for shift in (0, 5):
            got = _pack_dev(mdt, t, src, 32, 1, 0, -1, shift)
            assert first_diff(got, full) is None, (spec, shift)
        got = _pack_dev(mdt, t, src, 32, 1, a["size"] // 3, 11, 3)
        assert first_diff(got, o.pack(host, 32, 1, a["size"] // 3, 11)) is None, spec
        canary = np.full(size, 0x5A, np.uint8)
        exp = canary.copy()
        o.unpack(full, exp, 32, 1)
        dst = to_dev(canary)
        mdt.mdt_unpack(to_dev(full).data_ptr(), full.size, dst.data_ptr() + 32, 1, t, 0)
        assert first_diff(to_host(dst), exp) is None, spec


def test_darray_midsize(mdt):
    """Block-cyclic 3-D distributions of a 96 x 80 x 64 float64 array (and
    particle records on a 2-D grid) over several ranks: many tiles, ragged
    ends, chunked partial packs and unpacks."""
    D = ("basic", "DOUBLE")
    gs = [96, 80, 64]
    cases = [("darray", 8, r, gs, ["cyclic", "block", "cyclic"], [4, None, 8], [2, 2, 2], "C", D) for r in (0, 5, 7)]
    cases += [("darray", 6, r, gs, ["block", "cyclic", "none"], [None, 3, None], [3, 2, 1], "F", D) for r in (1, 4)]
    cases += [("darray", 4, 3, [300, 250], ["cyclic", "cyclic"], [7, None], [2, 2], "C", inputs.particle_struct())]
    for i, spec in enumerate(cases):
        note(f"darray midsize {i}: {spec[1:8]}")
        o = obuild(spec)
        _layout_case(mdt, spec, 1, o.attrs()["extent"], 0, seed=700 + i, chunk=(1 << 15) + 7)
