"""Host logic of libmdt (no GPU needed): constructors, attributes, commit,
and the segment queries mdt_type_iov_len / mdt_type_iov, compared with the
oracle on the same specs -- random tiny types of every constructor and the
workload layouts at full size.  Also checks that regular layouts compile to
a description whose size does not grow with the segment count."""
import numpy as np
import pytest

import bruteforce as bf
from oracle import build_type as obuild
from paper_2402_12274_amd import inputs
from typegen import tiny_specs

mdt = pytest.importorskip("paper_2402_12274_amd.mdt")


def _cmp_attrs(t, o):
    a = o.attrs()
    assert t.size() == a["size"]
    assert t.extent() == (a["lb"], a["extent"])
    assert t.true_extent() == (a["true_lb"], a["true_extent"])


def _cmp_segments(t, o, probe_all=True):
    nseg, size = o.iov_len(-1)
    assert t.iov_len(-1) == (nseg, size)
    ob, ol = o.iov(0, nseg)
    tb, tl = t.iov(0, nseg + 2)
    assert np.array_equal(tb, ob) and np.array_equal(tl, ol)
    if probe_all:
        for mb in range(0, size + 2):
            assert t.iov_len(mb) == o.iov_len(mb), mb
    else:
        g = np.random.Generator(np.random.PCG64(nseg))
        for mb in list(g.integers(0, size + 1, 200)) + [0, size - 1, size, size + 1]:
            assert t.iov_len(int(mb)) == o.iov_len(int(mb)), mb
    for off in (0, 1, nseg // 2, max(nseg - 1, 0), nseg, nseg + 3):
        for m in (0, 1, 3, 17):
            b1, l1 = t.iov(off, m)
            b2, l2 = o.iov(off, m)
            assert np.array_equal(b1, b2) and np.array_equal(l1, l2)


SPECS = tiny_specs(4242, 200)


@pytest.mark.parametrize("i", range(len(SPECS)))
def test_random_types_match_oracle(i):
    spec = SPECS[i]
    t = mdt.build_type(spec)
    o = obuild(spec)
    _cmp_attrs(t, o)
    _cmp_segments(t, o)


# Types whose element is one run that does not start at displacement 0:
# touching blocks collapse into a single run at their first block's offset
# (a layout that moves as one contiguous copy), alone and repeated.
I32 = ("basic", "INT32")
ONE_RUN_AT_OFFSET = [
    ("hindexed", [1, 1], [-19, -15], I32),
    ("contiguous", 2, ("hindexed", [1, 1], [-19, -15], I32)),
    ("hvector", 1, 2, 38, ("hindexed", [1, 1], [-19, -15], I32)),
    ("contiguous", 3, ("hindexed", [1, 1, 1], [5, 9, 13], I32)),
    ("contiguous", 2, ("struct", [1, 1], [16, 24], [inputs.DOUBLE, inputs.DOUBLE])),
    ("contiguous", 2, ("indexed", [2, 1], [3, 5], I32)),
]


@pytest.mark.parametrize("spec", ONE_RUN_AT_OFFSET)
def test_one_run_at_an_offset_matches_oracle(spec):
    # regression: the segment of such a type came out at twice its offset
    t = mdt.build_type(spec)
    o = obuild(spec)
    _cmp_attrs(t, o)
    _cmp_segments(t, o)
    for count in (0, 2, 3):
        n = o.iov_len(-1, count)[0]
        assert t.iov_len(-1, count) == o.iov_len(-1, count)
        b1, l1 = t.iov(0, n + 1, count)
        b2, l2 = o.iov(0, n + 1, count)
        assert np.array_equal(b1, b2) and np.array_equal(l1, l2), count


def test_workload_types_match_oracle():
    specs = [inputs.vector_small(), inputs.particle_struct()]
    specs += [s for _, s in inputs.halo_faces(512)]
    for spec in specs:
        t = mdt.build_type(spec)
        o = obuild(spec)
        _cmp_attrs(t, o)
        _cmp_segments(t, o, probe_all=False)


def test_hindexed_workload_matches_oracle():
    lens, disps = inputs.hindexed_blocks(nblocks=100_000, span=1 << 26, seed=7)
    spec = inputs.hindexed_type(lens, disps)
    t = mdt.build_type(spec)
    o = obuild(spec)
    _cmp_attrs(t, o)
    _cmp_segments(t, o, probe_all=False)


def test_worked_example_through_library():
    import json
    import os

    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "typeiov_example.json")))
    t = mdt.build_type(g["spec"])
    assert t.iov_len(g["max_iov_bytes"]) == (g["iov_len"], g["actual_iov_bytes"])
    b, ln = t.iov(0, 4)
    assert b.tolist() == g["iov_base"] and ln.tolist() == g["iov_len_each"]
    assert t.extent() == (g["lb"], g["extent"])
    assert t.true_extent() == (g["true_lb"], g["true_extent"])


def test_errors():
    D = inputs.DOUBLE
    t = mdt.build_type(("vector", 4, 1, 2, D))
    with pytest.raises(mdt.MdtError) as e:
        t.iov_len(-2)
    assert e.value.code == mdt.ERR_ARG
    u = mdt.build_type(("vector", 4, 1, 2, D), commit=False)
    with pytest.raises(mdt.MdtError) as e:
        u.iov_len(-1)
    assert e.value.code == mdt.ERR_TYPE
    assert u.size() == 32  # attributes work before commit
    for bad in [("subarray", [4], [5], [0], "C", D), ("subarray", [4], [2], [3], "C", D),
                ("vector", -1, 1, 1, D), ("hindexed", [1, -1], [0, 8], D),
                ("vector", 2, 1, 2 ** 62, ("vector", 2, 1, 2 ** 62, D))]:
        with pytest.raises(mdt.MdtError) as e:
            mdt.build_type(bad)
        assert e.value.code == mdt.ERR_ARG
    # freed handle
    h = mdt._P(t.handle)
    mdt.check(mdt.lib().mdt_type_free(mdt.C.byref(h)))
    t.owned = False
    assert h.value is None


def test_children_outlive_free():
    D = inputs.DOUBLE
    c = mdt.build_type(("vector", 3, 1, 2, D), commit=False)
    out = mdt._P()
    mdt.check(mdt.lib().mdt_type_contiguous(4, c.h, mdt.C.byref(out)))
    parent = mdt.Type(out.value)
    del c  # frees the caller's reference to the child
    parent.commit()
    assert parent.size() == 96
    # each copy's last element ends where the next copy's first begins, so
    # 12 runs merge into 9 segments
    assert parent.iov_len(-1) == obuild(("contiguous", 4, ("vector", 3, 1, 2, D))).iov_len(-1) == (9, 96)


def test_regular_layout_description_is_constant_size():
    # The YZ-surface argument: the segment count grows as N^2 but the
    # compiled description does not (no per-segment table is built).
    import ctypes

    for n in (64, 256, 1024):
        t = mdt.build_type(("subarray", [n, n, n], [n, n, 1], [0, 0, 0], "C", inputs.DOUBLE))
        assert t.iov_len(-1) == (n * n, n * n * 8)
    # the face of a 1024^3 array (1M segments) commits and answers a query
    # deep inside it by position arithmetic
    b, ln = t.iov(n * n - 1, 1)
    assert b[0] == ((n - 1) * n * n + (n - 1) * n) * 8 and ln[0] == 8
    assert ctypes.sizeof(mdt.Iov) == 16


def test_layout_info_reports_the_program():
    # the compiled program's shape, and which record tables the kernels use
    c = mdt.build_type(("contiguous", 1 << 20, inputs.DOUBLE)).layout_info()
    assert c["kind"] == 1 and c["runs"] == 1 and c["records"] == 0
    # a face of a 512^3 array: one shape over 510^2 runs, device tables of
    # constant size whatever the segment count
    f = mdt.build_type(inputs.halo_face(512, 1, 2, "lo")).layout_info()
    assert f["kind"] == 2 and f["runs"] == 510 * 510 and f["records"] == 0 and f["device_bytes"] < 4096
    # particle records: 33 packed bytes every 40, chunk and dword tables
    p = mdt.build_type(inputs.particle_struct()).layout_info()
    assert (p["records"], p["record_bytes"], p["record_stride"], p["pack_table"], p["unpack_table"]) == \
        (1, 33, 40, 2, 2)
    # irregular blocks: a group table, O(blocks) device bytes
    lens, disps = inputs.hindexed_blocks(nblocks=5000, span=1 << 20, seed=2)
    h = mdt.build_type(inputs.hindexed_type(lens, disps)).layout_info()
    assert h["kind"] == 3 and h["groups"] >= 4000 and h["device_bytes"] >= 5000 * 16
    # an uncommitted handle has no program
    import ctypes

    raw = ctypes.c_void_p()
    assert mdt._lib.mdt_type_contiguous(3, mdt.basic("DOUBLE").h, ctypes.byref(raw)) == 0
    info = mdt.LayoutInfo()
    assert mdt._lib.mdt_type_layout_info(raw, ctypes.byref(info)) == mdt.ERR_TYPE
    assert mdt._lib.mdt_type_free(ctypes.byref(raw)) == 0


def test_darray_matches_oracle():
    """Distributed arrays through the library (built from subarray, or from
    hindexed and resized per dimension) against the oracle's enumeration."""
    from typegen import darray_specs

    for spec in darray_specs(77, 150):
        t = mdt.build_type(spec)
        o = obuild(spec)
        _cmp_attrs(t, o)
        _cmp_segments(t, o, probe_all=False)


def test_darray_errors():
    D = ("basic", "DOUBLE")
    bad = [
        ("darray", 4, 0, [8, 8], ["block", "block"], [None, None], [2, 3], "C", D),
        ("darray", 4, -1, [8, 8], ["block", "block"], [None, None], [2, 2], "C", D),
        ("darray", 2, 0, [8], ["none"], [None], [2], "C", D),
        ("darray", 2, 0, [8], ["block"], [3], [2], "C", D),
        ("darray", 2, 0, [8], ["cyclic"], [0], [2], "C", D),
        ("darray", 2, 0, [8], ["diagonal"], [None], [2], "C", D),
        ("darray", 2, 0, [0], ["block"], [None], [2], "C", D),
        ("darray", 2, 0, [8], ["block"], [None], [2], "Z", D),
    ]
    for spec in bad:
        with pytest.raises(mdt.MdtError) as e:
            mdt.build_type(spec)
        assert e.value.code == mdt.ERR_ARG, spec


def _norm(spec):
    """A spec with every array as a plain list of ints (for comparison)."""
    if isinstance(spec, tuple):
        return tuple(_norm(x) for x in spec)
    if isinstance(spec, (list, np.ndarray)):
        return [_norm(x) for x in list(spec)]
    if isinstance(spec, (np.integer,)):
        return int(spec)
    return spec


def test_envelope_and_contents_round_trip():
    """Type envelope and contents give back the constructor call each type
    was made with, recursively, for every constructor (random tiny types,
    distributed arrays, the workload types); the rebuilt type has the same
    attributes and segments."""
    from typegen import darray_specs

    specs = list(SPECS[:120]) + darray_specs(5, 40) + [inputs.vector_small(), inputs.particle_struct()]
    specs += [s for _, s in inputs.halo_faces(64)]
    specs += [("indexed_block", 3, [4, 0, 9], ("basic", "INT16")), ("hindexed_block", 2, [16, -8], ("basic", "INT32")),
              ("dup", ("vector", 3, 2, 4, ("basic", "DOUBLE")))]
    for spec in specs:
        t = mdt.build_type(spec)
        back = mdt.spec_of(t)
        assert _norm(back) == _norm(spec), (spec, back)
        t2 = mdt.build_type(back)
        assert t2.size() == t.size() and t2.extent() == t.extent() and t2.true_extent() == t.true_extent()
        n = t.iov_len(-1)[0]
        b1, l1 = t.iov(0, n)
        b2, l2 = t2.iov(0, n)
        assert np.array_equal(b1, b2) and np.array_equal(l1, l2)


def test_envelope_of_predefined_and_errors():
    import ctypes as C

    comb, ni, na, nt = mdt.envelope(mdt.Type(mdt.lib().mdt_basic(mdt.BASIC_CODES["DOUBLE"]), owned=False))
    assert (comb, ni, na, nt) == ("named", 0, 0, 0)
    t = mdt.build_type(("vector", 3, 2, 4, ("basic", "DOUBLE")))
    ints = (C.c_int64 * 3)()
    kids = (C.c_void_p * 1)()
    # too small an integer array: nothing written
    assert mdt.lib().mdt_type_get_contents(t.h, 2, 0, 1, ints, None, kids) == mdt.ERR_ARG
    assert list(ints) == [0, 0, 0] and kids[0] is None
    d = mdt.Type(mdt.lib().mdt_basic(mdt.BASIC_CODES["DOUBLE"]), owned=False)
    assert mdt.lib().mdt_type_get_contents(d.h, 0, 0, 0, None, None, None) == mdt.ERR_ARG


def test_darray_cyclic_is_constant_size():
    """A cyclic dimension is one strided vector, not a list of its blocks:
    a 10^9-element cyclic(1) array over 2 processes builds instantly into a
    one-group program, with the closed-form size, bounds and segments."""
    g = 10 ** 9
    t = mdt.build_type(("darray", 2, 1, [g], ["cyclic"], [None], [2], "C", ("basic", "DOUBLE")))
    assert t.size() == (g // 2) * 8
    assert t.extent() == (0, g * 8)
    assert t.true_extent() == (8, (g - 1) * 8 - 8 + 8)
    info = t.layout_info()
    assert info["groups"] == 1 and info["device_bytes"] < 1 << 14
    b, ln = t.iov(0, 3)
    assert list(b) == [8, 24, 40] and list(ln) == [8, 8, 8]
    # a partial last block: 10 elements, cyclic(3) over 2 -> rank 0 owns 0-2, 6-8; rank 1 owns 3-5, 9
    t = mdt.build_type(("darray", 2, 1, [10], ["cyclic"], [3], [2], "C", ("basic", "INT32")))
    b, ln = t.iov(0, 4)
    assert list(b) == [12, 36] and list(ln) == [12, 4]


def _cmp_segments_count(t, o, count, probe_all=True):
    nseg, size = o.iov_len(-1, count)
    assert t.iov_len(-1, count) == (nseg, size)
    ob, ol = o.iov(0, nseg, count)
    tb, tl = t.iov(0, nseg + 2, count)
    assert np.array_equal(tb, ob) and np.array_equal(tl, ol), count
    budgets = range(0, size + 2) if probe_all else \
        [int(x) for x in np.random.Generator(np.random.PCG64(nseg)).integers(0, size + 1, 200)] + [0, size - 1, size]
    for mb in budgets:
        assert t.iov_len(mb, count) == o.iov_len(mb, count), (count, mb)
    for off in (0, 1, nseg // 2, max(nseg - 1, 0), nseg, nseg + 3):
        for m in (0, 1, 3, 17):
            b1, l1 = t.iov(off, m, count)
            b2, l2 = o.iov(off, m, count)
            assert np.array_equal(b1, b2) and np.array_equal(l1, l2), (count, off, m)


@pytest.mark.parametrize("i", range(0, len(SPECS), 3))
def test_iov_count_matches_oracle(i):
    # the count form of the segment queries, on random types (merge-free
    # layouts and those with a merged-segment table) and counts 0..4
    spec = SPECS[i]
    t = mdt.build_type(spec)
    o = obuild(spec)
    for count in (0, 1, 2, 4):
        _cmp_segments_count(t, o, count)


def test_iov_count_boundary_merges_and_errors():
    D = inputs.DOUBLE
    cases = [("resized", 0, 12, ("vector", 2, 1, 2, ("basic", "INT32"))),   # last run touches the next element
             inputs.vector_small(),                                          # ditto (extent = last run's end)
             ("contiguous", 3, D),                                           # one segment for every count
             ("resized", 0, 24, ("contiguous", 3, D)),                       # elements touch: one segment
             ("resized", 0, 32, ("contiguous", 3, D)),                       # a gap between elements
             ("resized", -8, 16, ("hindexed", [1, 1], [8, -8], D)),          # map order descending
             inputs.particle_struct()]
    for spec in cases:
        t = mdt.build_type(spec)
        o = obuild(spec)
        for count in (0, 1, 2, 3, 17):
            _cmp_segments_count(t, o, count)
    t = mdt.build_type(inputs.vector_small())
    with pytest.raises(mdt.MdtError) as e:
        t.iov_len(-1, -1)
    assert e.value.code == mdt.ERR_ARG
    with pytest.raises(mdt.MdtError) as e:
        t.iov(0, 1, 1 << 62)
    assert e.value.code == mdt.ERR_COUNT
    # the worked example's halo face over a count: the library's counted
    # segments at full size (sampled budgets)
    spec = inputs.halo_face(512, 1, 2, "lo")
    _cmp_segments_count(mdt.build_type(spec), obuild(spec), 2, probe_all=False)
