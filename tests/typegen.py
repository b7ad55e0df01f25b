"""Seeded random generator of tiny, arbitrarily nested type specs (tests only).

Covers every constructor, negative strides and displacements, zero block
lengths, resized types with shifted or shrunk extents, mixed-size struct
members and C/Fortran subarrays.  Types are kept small enough for the
brute-force enumerator.
"""
from __future__ import annotations

import numpy as np

from bruteforce import typemap

BASICS = ["BYTE", "CHAR", "INT16", "INT32", "FLOAT", "DOUBLE", "INT64"]


def _basic(g):
    return ("basic", BASICS[int(g.integers(0, len(BASICS)))])


def random_spec(g: np.random.Generator, depth: int = 0, allow_overlap: bool = True):
    if depth >= 3 or g.random() < 0.25 + 0.15 * depth:
        return _basic(g)
    child = random_spec(g, depth + 1, allow_overlap)
    k = int(g.integers(0, 12))
    small = lambda lo, hi: int(g.integers(lo, hi + 1))  # noqa: E731
    if k == 0:
        return ("contiguous", small(0, 4), child)
    if k == 1:
        st = small(-4, 6) if allow_overlap else small(2, 6)
        return ("vector", small(0, 4), small(0, 3), st, child)
    if k == 2:
        st = small(-40, 60) if allow_overlap else small(40, 80)
        return ("hvector", small(0, 4), small(0, 3), st, child)
    if k in (3, 4):
        n = small(0, 4)
        bls = [small(0, 3) for _ in range(n)]
        disps = [small(-8, 12) if k == 3 else small(-64, 96) for _ in range(n)]
        return ("indexed" if k == 3 else "hindexed", bls, disps, child)
    if k in (5, 6):
        n = small(0, 4)
        disps = [small(-8, 12) if k == 5 else small(-64, 96) for _ in range(n)]
        return ("indexed_block" if k == 5 else "hindexed_block", small(0, 3), disps, child)
    if k == 7:
        n = small(1, 3)
        kids = [child] + [random_spec(g, depth + 1, allow_overlap) for _ in range(n - 1)]
        bls = [small(0, 3) for _ in range(n)]
        disps = sorted(small(-16, 64) for _ in range(n))
        return ("struct", bls, disps, kids)
    if k == 8:
        nd = small(1, 3)
        sizes = [small(1, 5) for _ in range(nd)]
        subs = [small(0 if g.random() < 0.05 else 1, s) for s in sizes]
        starts = [small(0, s - u) for s, u in zip(sizes, subs)]
        return ("subarray", sizes, subs, starts, "C" if g.random() < 0.6 else "F", child)
    if k == 9:
        return ("resized", small(-16, 16), small(0, 48) if g.random() < 0.9 else small(-24, -1), child)
    if k == 10:
        return ("dup", child)
    return ("contiguous", small(1, 3), child)


def tiny_specs(seed: int, n: int, max_entries: int = 600, allow_overlap: bool = True):
    """``n`` random specs whose typemap has at most ``max_entries`` entries and
    whose bytes span at most 64 KiB."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    while len(out) < n:
        spec = random_spec(g, 0, allow_overlap)
        tm = typemap(spec)
        if len(tm.entries) > max_entries:
            continue
        if tm.true_ub - tm.true_lb > 65536 or abs(tm.extent) > 65536:
            continue
        out.append(spec)
    return out


def buffer_for(tm, count: int, pad: int = 16):
    """(size, origin) of a host buffer covering every byte (count x type)
    touches, with ``pad`` guard bytes on both sides."""
    if not tm.entries or count == 0:
        return 2 * pad, pad
    lo = min(r * tm.extent + tm.true_lb for r in range(count))
    hi = max(r * tm.extent + tm.true_ub for r in range(count))
    return hi - lo + 2 * pad, pad - lo


def darray_specs(seed: int, n: int, max_g: int = 12):
    """Random distributed-array specs: 1-3 dimensions, every distribution,
    default and explicit distribution arguments, both orders, basic and
    derived (gapped) element types, any rank of the process grid."""
    g = np.random.Generator(np.random.PCG64(seed))
    elems = [("basic", "DOUBLE"), ("basic", "INT32"), ("basic", "BYTE"), ("basic", "INT16"),
             ("vector", 2, 1, 3, ("basic", "INT32")), ("contiguous", 3, ("basic", "INT16"))]
    out = []
    while len(out) < n:
        nd = int(g.integers(1, 4))
        gs = [int(g.integers(1, max_g + 1)) for _ in range(nd)]
        ds, da, ps = [], [], []
        for k in range(nd):
            d = ["none", "block", "cyclic"][int(g.integers(0, 3))]
            p = 1 if d == "none" else int(g.integers(1, 5))
            a = None
            if d == "block" and g.random() < 0.5:
                a = -(-gs[k] // p) + int(g.integers(0, 3))  # any block size that covers the dimension
            elif d == "cyclic" and g.random() < 0.6:
                a = int(g.integers(1, 5))
            ds.append(d)
            da.append(a)
            ps.append(p)
        size = int(np.prod(ps))
        rank = int(g.integers(0, size))
        order = "C" if g.random() < 0.5 else "F"
        elem = elems[int(g.integers(0, len(elems)))]
        out.append(("darray", size, rank, gs, ds, da, ps, order, elem))
    return out
