"""Pins of the oracle against facts it does not compute itself.

- the worked example of the Derived Datatypes section (values derived by
  hand, stored under tests/golden/ with their citation);
- the YZ-surface segment count of the same section;
- closed forms of the small-vector, halo-face and particle-record layouts;
- library routines that reduce to special cases: numpy slicing (subarray,
  C and Fortran order), numpy strided views (vector), numpy structured
  dtypes with C alignment (struct padding and field extraction), memcpy
  (contiguous);
- brute-force typemap enumeration on random tiny types (every constructor);
- invariants (chunked partial packs concatenate, unpack inverts pack,
  count-fold streams concatenate, dup and equivalent constructions agree).
"""
import json
import os

import numpy as np
import pytest

import bruteforce as bf
import oracle
from oracle import OracleError, build_type
from paper_2402_12274_amd import inputs
from typegen import buffer_for, tiny_specs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------------------
# worked example


def test_worked_example_typeiov():
    g = _load("typeiov_example.json")
    t = build_type(g["spec"])
    a = t.attrs()
    assert a["size"] == g["size"]
    assert a["lb"] == g["lb"] and a["extent"] == g["extent"]
    assert a["true_lb"] == g["true_lb"] and a["true_extent"] == g["true_extent"]
    assert t.iov_len(g["max_iov_bytes"]) == (g["iov_len"], g["actual_iov_bytes"])
    base, ln = t.iov(g["iov_offset"], g["max_iov_len"])
    assert base.tolist() == g["iov_base"]
    assert ln.tolist() == g["iov_len_each"]
    assert hex(base[0]) == "0x11e6380c0"


def test_yz_surface_segment_count():
    for case in _load("yz_surface.json")["cases"]:
        nz, ny, nx = case["dims"]
        spec = ("subarray", [nz, ny, nx], [nz, ny, 1], [0, 0, case["x"]], "C", ("basic", case["elem"]))
        t = build_type(spec)
        base, ln = t.iov(0, case["segments"] + 5)
        assert t.num_segments() == case["segments"] == len(base)
        assert set(ln.tolist()) == {case["seg_bytes"]}


# ---------------------------------------------------------------------------
# closed forms of the workload layouts


def test_small_vector_closed_form():
    t = build_type(inputs.vector_small())
    a = t.attrs()
    assert a["size"] == 8192
    assert a["extent"] == a["true_extent"] == 16376
    assert t.num_segments() == 1024
    base, ln = t.iov(0, 1024)
    assert (base == 16 * np.arange(1024)).all() and (ln == 8).all()
    assert t.iov_len(-1) == (1024, 8192)
    assert t.iov_len(4096) == (512, 4096)
    assert t.iov_len(4100) == (512, 4096)
    assert t.iov(512, 3)[0][0] == 8192


@pytest.mark.parametrize("w", [1, 4])
def test_halo_face_closed_forms(w):
    n = 64
    m = n - 2 * w
    for label, spec in inputs.halo_faces(n, (w,)):
        t = build_type(spec)
        dim = int(label.split("-")[1][1])
        a = t.attrs()
        assert a["size"] == m * m * w * 8
        assert a["lb"] == 0 and a["extent"] == n ** 3 * 8
        nseg = t.num_segments()
        base, ln = t.iov(0, nseg)
        if dim == 2:   # fastest dim fixed: one w-wide block per (z, y)
            assert nseg == m * m and set(ln.tolist()) == {8 * w}
        elif dim == 1:  # one interior row per (z, y in face)
            assert nseg == m * w and set(ln.tolist()) == {8 * m}
        else:           # slowest fixed: interior rows of each plane
            assert nseg == w * m and set(ln.tolist()) == {8 * m}


def test_halo_face_full_size_w1():
    # 512^3 array: most-fragmented face has 510^2 segments of 8 B
    t = build_type(inputs.halo_face(512, 1, 2, "lo"))
    assert t.num_segments() == 260100
    assert t.attrs()["size"] == 2080800
    t4 = build_type(inputs.halo_face(512, 4, 2, "hi"))
    assert t4.num_segments() == 254016
    assert t4.attrs()["size"] == 8128512


def test_particle_struct_matches_numpy_aligned_dtype():
    t = build_type(inputs.particle_struct())
    a = t.attrs()
    dt = np.dtype({"names": ["i", "d", "c"], "formats": ["<i4", ("<f8", 3), "S5"]}, align=True)
    assert dt.itemsize == 40 and dt.fields["d"][1] == 8 and dt.fields["c"][1] == 32
    assert a["size"] == 33 and a["extent"] == dt.itemsize and a["true_extent"] == 37
    base, ln = t.iov(0, 10)
    assert list(zip(base.tolist(), ln.tolist())) == [(0, 4), (8, 29)]
    count = 1000
    buf = inputs.random_bytes(count * 40, seed=5)
    rec = buf.reshape(count, 40)
    expect = np.concatenate([rec[:, 0:4], rec[:, 8:37]], axis=1).ravel()
    got = t.pack(buf, 0, count)
    assert np.array_equal(got, expect)
    # 1 MiB-style partial packs: chunks concatenate to the full pack
    parts = [t.pack(buf, 0, count, off, 997) for off in range(0, count * 33, 997)]
    assert np.array_equal(np.concatenate(parts), expect)


# ---------------------------------------------------------------------------
# library routines for special cases


@pytest.mark.parametrize("order", ["C", "F"])
def test_subarray_matches_numpy_slicing(order):
    g = np.random.Generator(np.random.PCG64(11))
    for _ in range(25):
        nd = int(g.integers(1, 5))
        sizes = [int(g.integers(1, 9)) for _ in range(nd)]
        subs = [int(g.integers(1, s + 1)) for s in sizes]
        starts = [int(g.integers(0, s - u + 1)) for s, u in zip(sizes, subs)]
        elem = ["DOUBLE", "INT32", "INT16", "BYTE"][int(g.integers(0, 4))]
        es = bf.SIZES[elem]
        t = build_type(("subarray", sizes, subs, starts, order, ("basic", elem)))
        total = int(np.prod(sizes))
        buf = inputs.random_bytes(total * es, seed=int(g.integers(0, 1 << 30)))
        elems = buf.reshape(total, es)
        # numpy's own row-/column-major indexing of the full array
        lin = np.arange(total).reshape(sizes, order=order)
        sl = tuple(slice(s, s + u) for s, u in zip(starts, subs))
        picked = lin[sl].ravel(order=order)
        expect = elems[picked].ravel()
        assert np.array_equal(t.pack(buf, 0, 1), expect)
        a = t.attrs()
        assert a["lb"] == 0 and a["extent"] == total * es


def test_vector_matches_numpy_strided_view():
    g = np.random.Generator(np.random.PCG64(12))
    for _ in range(30):
        n, bl, st = int(g.integers(1, 40)), int(g.integers(1, 5)), int(g.integers(1, 9))
        st = max(st, bl)
        t = build_type(("vector", n, bl, st, inputs.DOUBLE))
        buf = inputs.random_bytes(((n - 1) * st + bl) * 8, seed=int(g.integers(0, 1 << 30)))
        f = buf.view(np.float64)
        view = np.lib.stride_tricks.as_strided(f, shape=(n, bl), strides=(st * 8, 8))
        assert np.array_equal(t.pack(buf, 0, 1), np.ascontiguousarray(view).view(np.uint8).ravel())
        assert t.attrs()["extent"] == ((n - 1) * st + bl) * 8


def test_contiguous_packs_like_memcpy():
    buf = inputs.random_bytes(1 << 16, seed=3)
    t = build_type(("contiguous", 1 << 13, inputs.DOUBLE))
    assert np.array_equal(t.pack(buf, 0, 1), buf)
    assert t.num_segments() == 1
    assert np.array_equal(t.pack(buf, 0, 1, 1000, 12345), buf[1000:13345])
    t2 = build_type(("contiguous", 100, inputs.BYTE))
    assert np.array_equal(t2.pack(buf, 0, 300), buf[:30000])


# ---------------------------------------------------------------------------
# brute force on random tiny types


SPECS = tiny_specs(20240219, 160)


def _attrs_bf(tm):
    return dict(size=tm.size, lb=tm.lb, ub=tm.ub, true_lb=tm.true_lb, true_ub=tm.true_ub)


@pytest.mark.parametrize("i", range(len(SPECS)))
def test_oracle_vs_bruteforce(i):
    spec = SPECS[i]
    tm = bf.typemap(spec)
    t = build_type(spec)
    a = t.attrs()
    assert {k: a[k] for k in ("size", "lb", "ub", "true_lb", "true_ub")} == _attrs_bf(tm), spec
    assert a["entries"] == len(tm.entries)
    segs = bf.segments(tm)
    assert t.num_segments() == len(segs)
    b, ln = t.iov(0, len(segs) + 3)
    assert list(zip(b.tolist(), ln.tolist())) == segs
    for off in range(0, len(segs) + 2):
        for m in (0, 1, 2, 5):
            b, ln = t.iov(off, m)
            assert list(zip(b.tolist(), ln.tolist())) == bf.iov(tm, off, m)
    for mb in [-1] + list(range(0, tm.size + 2)):
        assert t.iov_len(mb) == bf.iov_len(tm, mb), (spec, mb)
    for count in (0, 1, 3):
        size, origin = buffer_for(tm, count)
        buf = inputs.random_bytes(size, seed=i * 7 + count)
        total = count * tm.size
        full = bf.pack(tm, buf, origin, count)
        assert np.array_equal(t.pack(buf, origin, count), full)
        for off in sorted({0, 1, total // 3, total // 2, max(total - 1, 0), total, total + 5}):
            for mb in (-1, 0, 1, 7, total):
                assert np.array_equal(t.pack(buf, origin, count, off, mb),
                                      bf.pack(tm, buf, origin, count, off, mb)), (spec, count, off, mb)
        if bf.overlaps(tm, count):
            with pytest.raises(OracleError) as e:
                t.unpack(full, np.zeros_like(buf), origin, count)
            assert e.value.code == oracle.oracle.ERR_OVERLAP
        else:
            dst = np.full_like(buf, 0xA5)
            exp = dst.copy()
            bf.unpack(tm, full, exp, origin, count)
            assert t.unpack(full, dst, origin, count) == total
            assert np.array_equal(dst, exp)
            if total > 2:
                # partial unpack at an offset leaves everything else alone
                dst2 = np.full_like(buf, 0x3C)
                exp2 = dst2.copy()
                lo, hi = total // 3, total - 1
                bf.unpack(tm, full[lo:hi], exp2, origin, count, lo)
                t.unpack(full[lo:hi], dst2, origin, count, lo)
                assert np.array_equal(dst2, exp2)


@pytest.mark.parametrize("i", range(0, len(SPECS), 2))
def test_oracle_iov_count_vs_bruteforce(i):
    # segment queries over count consecutive elements: the brute-force list
    # of count shifted copies, merged where one element's last run touches
    # the next element's first
    spec = SPECS[i]
    tm = bf.typemap(spec)
    t = build_type(spec)
    for count in (0, 2, 3):
        rt = bf.repeat(tm, count)
        segs = bf.segments(rt)
        assert t.num_segments(count) == len(segs), (spec, count)
        b, ln = t.iov(0, len(segs) + 3, count)
        assert list(zip(b.tolist(), ln.tolist())) == segs, (spec, count)
        for off in range(0, len(segs) + 2, max(1, len(segs) // 7)):
            for m in (0, 1, 3):
                b, ln = t.iov(off, m, count)
                assert list(zip(b.tolist(), ln.tolist())) == bf.iov(rt, off, m), (spec, count, off, m)
        for mb in [-1] + list(range(0, rt.size + 2)):
            assert t.iov_len(mb, count) == bf.iov_len(rt, mb), (spec, count, mb)


def test_iov_count_closed_forms():
    # worked by hand: resized(vector(2, 1, 2, INT32), lb 0, extent 12) puts
    # element r's runs at 12r and 12r + 8 (4 bytes each): the second run of
    # one element ends where the next element's first begins, so k elements
    # give 1 + k segments: 4 bytes, k - 1 merged 8-byte runs, 4 bytes
    spec = ("resized", 0, 12, ("vector", 2, 1, 2, ("basic", "INT32")))
    t = build_type(spec)
    for k in (1, 2, 3, 7):
        assert t.num_segments(k) == 1 + k
        b, ln = t.iov(0, 100, k)
        exp = [(0, 4)] + [(12 * r + 8, 8) for r in range(k - 1)] + [(12 * (k - 1) + 8, 4)]
        assert list(zip(b.tolist(), ln.tolist())) == exp
        # byte budgets: whole segments only (the merged run spans bytes 4..12)
        assert t.iov_len(11, k) == ((1, 4) if k > 1 else (2, 8))
        if k > 2:
            assert t.iov_len(12, k) == (2, 12) and t.iov_len(19, k) == (2, 12) and t.iov_len(20, k) == (3, 20)
    # a contiguous type: all elements form one segment
    c = build_type(("contiguous", 3, ("basic", "DOUBLE")))
    assert t.num_segments(0) == 0 and c.num_segments(5) == 1
    assert [x.tolist() for x in c.iov(0, 4, 5)] == [[0], [120]]
    assert c.iov_len(119, 5) == (0, 0) and c.iov_len(120, 5) == (1, 120) and c.iov_len(-1, 5) == (1, 120)
    # the C1 vector: vector(1024, 1, 2, DOUBLE) has extent 16,376 and its
    # last run [16368, 16376) ends where the next element's first run
    # begins, so k elements give 1024k - (k - 1) segments, the merged ones
    # 16 bytes long
    v = build_type(("vector", 1024, 1, 2, ("basic", "DOUBLE")))
    assert v.num_segments(3) == 3070
    b, ln = v.iov(1022, 3, 3)
    assert b.tolist() == [16352, 16368, 16392] and ln.tolist() == [8, 16, 8]
    with pytest.raises(OracleError):
        v.iov_len(-1, -1)


# ---------------------------------------------------------------------------
# invariants and error rules


def test_invariants_on_random_types():
    specs = [s for s in tiny_specs(777, 120, allow_overlap=False) if not bf.overlaps(bf.typemap(s), 3)]
    assert len(specs) > 40
    for i, spec in enumerate(specs):
        t = build_type(spec)
        a = t.attrs()
        nseg = t.num_segments()
        _, ln = t.iov(0, nseg)
        assert int(ln.sum()) == a["size"]                       # sum of iov lengths = size
        prev = (0, 0)
        for mb in range(0, a["size"] + 1):
            k, act = t.iov_len(mb)
            assert k >= prev[0] and act >= prev[1]              # monotone
            assert act <= mb
            if k < nseg:
                assert mb < act + ln[k]                         # bisection: P_k <= mb < P_{k+1}
            prev = (k, act)
        tm = bf.typemap(spec)
        count = 3
        size, origin = buffer_for(tm, count)
        buf = inputs.random_bytes(size, seed=100 + i)
        full = t.pack(buf, origin, count)
        # pack(count) = concatenation of pack(1) at r * extent
        parts = [t.pack(buf, origin + r * a["extent"], 1) for r in range(count)]
        assert np.array_equal(full, np.concatenate(parts) if parts else full)
        # chunked partial packs (1 B, primes) concatenate to the full pack
        for step in (1, 3, 7, 13):
            ch = [t.pack(buf, origin, count, o, step) for o in range(0, len(full), step)]
            assert np.array_equal(np.concatenate(ch) if ch else full, full)
        # unpack(pack(x)) restores covered bytes and leaves the rest untouched
        dst = np.zeros_like(buf)
        t.unpack(full, dst, origin, count)
        covered = np.zeros(len(buf), bool)
        covered[origin + bf.stream_addrs(tm, count)] = True
        assert np.array_equal(dst[covered], buf[covered]) and not dst[~covered].any()
        # dup is the same type
        d = build_type(("dup", spec))
        assert np.array_equal(d.pack(buf, origin, count), full)


def test_subarray_equals_nested_hvectors():
    sizes, subs, starts = [7, 6, 9], [3, 4, 5], [2, 1, 3]
    E = 8
    sub = build_type(("subarray", sizes, subs, starts, "C", inputs.DOUBLE))
    row = ("contiguous", subs[2], inputs.DOUBLE)
    plane = ("hvector", subs[1], 1, sizes[2] * E, row)
    box = ("hvector", subs[0], 1, sizes[1] * sizes[2] * E, plane)
    disp = ((starts[0] * sizes[1] + starts[1]) * sizes[2] + starts[2]) * E
    nested = build_type(("hindexed", [1], [disp], box))
    buf = inputs.random_bytes(int(np.prod(sizes)) * E, seed=9)
    assert np.array_equal(sub.pack(buf, 0, 1), nested.pack(buf, 0, 1))
    assert sub.num_segments() == nested.num_segments() == subs[0] * subs[1]


def test_error_rules():
    D = inputs.DOUBLE
    t = build_type(("vector", 4, 1, 2, D))
    with pytest.raises(OracleError):
        t.iov_len(-2)                        # only -1 is special
    with pytest.raises(OracleError):
        t.iov(-1, 3)
    assert t.iov(4, 3)[0].size == 0          # offset past the end: nothing
    assert t.iov_len(2 ** 31 - 1) == (4, 32)  # INT_MAX: all segments
    buf = inputs.random_bytes(64, seed=1)
    assert t.pack(buf, 0, 1, 40, -1).size == 0   # offset beyond the stream
    with pytest.raises(OracleError):
        t.unpack(np.zeros(40, np.uint8), np.zeros(64, np.uint8), 0, 1)  # truncate
    with pytest.raises(OracleError) as e:
        t.unpack(np.zeros(9, np.uint8), np.zeros(64, np.uint8), 0, 1, 24)
    assert e.value.code == oracle.oracle.ERR_TRUNCATE
    for bad in [("subarray", [4], [5], [0], "C", D), ("subarray", [4], [2], [3], "C", D),
                ("subarray", [4], [-1], [0], "C", D), ("vector", -1, 1, 1, D), ("vector", 2, -1, 1, D),
                ("hindexed", [1, -1], [0, 8], D), ("vector", 2, 1, 2 ** 62, ("vector", 2, 1, 2 ** 62, D))]:
        with pytest.raises(OracleError):
            build_type(bad)
    # overlapping types pack but do not unpack
    ov = build_type(("hindexed", [2, 2], [0, 8], D))
    buf = inputs.random_bytes(32, seed=2)
    p = ov.pack(buf, 0, 1)
    assert np.array_equal(p, np.concatenate([buf[0:16], buf[8:24]]))
    with pytest.raises(OracleError) as e:
        ov.unpack(p, np.zeros(32, np.uint8), 0, 1)
    assert e.value.code == oracle.oracle.ERR_OVERLAP


def test_multithreaded_pack_equals_single():
    t = build_type(inputs.particle_struct())
    count = 70000
    buf = inputs.random_bytes(count * 40, seed=21)
    one = t.pack(buf, 0, count)
    assert np.array_equal(t.pack(buf, 0, count, nthreads=4), one)
    assert np.array_equal(t.pack(buf, 0, count, 123457, 1 << 20, nthreads=3), one[123457:123457 + (1 << 20)])


# ---------------------------------------------------------------------------
# distributed arrays: pinned by properties the definition implies, not by
# restating its ownership rule

def _darray_labels(spec):
    """Linear element indices that (1 x spec) packs, for an INT32 element:
    the buffer holds each element's own linear index."""
    _, size, rank, gs, ds, da, ps, order, _ = spec
    s = ("darray", size, rank, gs, ds, da, ps, order, ("basic", "INT32"))
    t = build_type(s)
    total = int(np.prod(gs))
    buf = np.arange(total, dtype=np.int32).view(np.uint8)
    return np.frombuffer(t.pack(buf, 0, 1).tobytes(), dtype=np.int32), t


def test_darray_ranks_partition_the_array():
    """Over all ranks of the grid every element is owned exactly once, and
    each rank lists its elements in increasing linear order (row-major for
    C, column-major for Fortran)."""
    from typegen import darray_specs

    for spec in darray_specs(31, 60):
        _, size, _, gs, ds, da, ps, order, _ = spec
        seen = []
        for r in range(size):
            lab, t = _darray_labels(("darray", size, r, gs, ds, da, ps, order, None))
            assert np.all(np.diff(lab) > 0), spec
            a = t.attrs()
            assert a["lb"] == 0 and a["extent"] == 4 * int(np.prod(gs))
            seen.append(lab)
        allv = np.sort(np.concatenate(seen))
        assert np.array_equal(allv, np.arange(int(np.prod(gs)))), spec


def test_darray_block_is_a_subarray():
    """With one grid coordinate per dimension (psizes all 1) a block or
    undistributed darray is the whole array, and a block distribution of
    one dimension over p processes gives p consecutive slabs in rank
    order."""
    for order in ("C", "F"):
        lab, _ = _darray_labels(("darray", 1, 0, [5, 3, 4], ["block", "none", "block"], [None] * 3, [1, 1, 1],
                                 order, None))
        lin = np.arange(60).reshape([5, 3, 4], order=order).ravel(order=order)
        assert np.array_equal(lab, lin)
    # slabs: the C-order rows of a 10 x 6 array over 4 processes (3, 3, 3, 1 rows)
    got = [_darray_labels(("darray", 4, r, [10, 6], ["block", "none"], [None, None], [4, 1], "C", None))[0]
           for r in range(4)]
    sub = [build_type(("subarray", [10, 6], [n, 6], [s, 0], "C", ("basic", "INT32")))
           for s, n in ((0, 3), (3, 3), (6, 3), (9, 1))]
    buf = np.arange(60, dtype=np.int32).view(np.uint8)
    for g_, s_ in zip(got, sub):
        assert np.array_equal(g_, np.frombuffer(s_.pack(buf, 0, 1).tobytes(), dtype=np.int32))


def test_darray_cyclic_matches_numpy_reshape():
    """Cyclic(k) over p processes when k*p divides the dimension: rank c owns
    column c of the (g/(k p), p, k) reshape of the index range; with a
    second, undistributed dimension the rows are those indices."""
    for g_, k, p in ((24, 2, 3), (12, 1, 4), (30, 5, 3), (8, 4, 2)):
        for c in range(p):
            lab, _ = _darray_labels(("darray", p, c, [g_], ["cyclic"], [k], [p], "C", None))
            assert np.array_equal(lab, np.arange(g_).reshape(g_ // (k * p), p, k)[:, c, :].ravel())
            lab, _ = _darray_labels(("darray", p, c, [g_, 5], ["cyclic", "none"], [k, None], [p, 1], "C", None))
            rows = np.arange(g_).reshape(g_ // (k * p), p, k)[:, c, :].ravel()
            assert np.array_equal(lab, (rows[:, None] * 5 + np.arange(5)[None, :]).ravel())


def test_darray_error_rules():
    D = ("basic", "DOUBLE")
    bad = [
        ("darray", 4, 0, [8, 8], ["block", "block"], [None, None], [2, 3], "C", D),  # grid of 6 != 4
        ("darray", 4, 4, [8, 8], ["block", "block"], [None, None], [2, 2], "C", D),  # rank out of range
        ("darray", 2, 0, [8], ["none"], [None], [2], "C", D),                        # none over 2
        ("darray", 2, 0, [8], ["block"], [3], [2], "C", D),                          # 3 * 2 < 8
        ("darray", 2, 0, [8], ["cyclic"], [0], [2], "C", D),                         # darg 0
        ("darray", 2, 0, [8], ["diagonal"], [None], [2], "C", D),                    # no such distribution
        ("darray", 2, 0, [0], ["block"], [None], [2], "C", D),                       # empty dimension
        ("darray", 2, 0, [8], ["block"], [None], [2], "Z", D),                       # order
    ]
    for spec in bad:
        with pytest.raises(OracleError):
            build_type(spec)


def test_darray_default_arguments():
    """The default distribution argument is 1 for cyclic and ceil(g / p)
    for block (MPI's defaults)."""
    for g_, p in ((10, 3), (7, 7), (9, 2), (1, 4)):
        for c in range(p):
            d, _ = _darray_labels(("darray", p, c, [g_], ["cyclic"], [None], [p], "C", None))
            e, _ = _darray_labels(("darray", p, c, [g_], ["cyclic"], [1], [p], "C", None))
            assert np.array_equal(d, e)
            d, _ = _darray_labels(("darray", p, c, [g_], ["block"], [None], [p], "C", None))
            e, _ = _darray_labels(("darray", p, c, [g_], ["block"], [-(-g_ // p)], [p], "C", None))
            assert np.array_equal(d, e)
