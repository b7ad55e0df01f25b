"""Brute-force typemap enumeration for tiny types (pins the oracle).

Builds the explicit typemap -- the ordered list of (displacement, size)
entries -- of a type spec by literally expanding every constructor, then
derives everything by definition: sizes and true bounds from the entry
list, segments by merging consecutive entries that touch, segment queries
by scanning that list, and pack/unpack by slicing bytes entry by entry.

It shares no code with the oracle (C) or with the product library; it is a
second, independent reading of the same definitions, written as list
manipulation instead of a streaming walk.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SIZES = {
    "BYTE": 1, "CHAR": 1, "INT8": 1, "UINT8": 1, "INT16": 2, "UINT16": 2,
    "INT32": 4, "UINT32": 4, "INT": 4, "FLOAT": 4, "INT64": 8, "UINT64": 8, "DOUBLE": 8,
}


@dataclass
class TM:
    entries: list          # [(disp, size)] in map order
    lb: int
    ub: int
    align: int
    explicit: bool

    @property
    def size(self):
        return sum(s for _, s in self.entries)

    @property
    def extent(self):
        return self.ub - self.lb

    @property
    def true_lb(self):
        return min((d for d, _ in self.entries), default=0)

    @property
    def true_ub(self):
        return max((d + s for d, s in self.entries), default=0)


def _place(copies, kind=None):
    """copies: list of (shift, TM).  Concatenate shifted entry lists."""
    entries = [(sh + d, s) for sh, c in copies for d, s in c.entries]
    if copies:
        lb = min(sh + c.lb for sh, c in copies)
        ub = max(sh + c.ub for sh, c in copies)
        align = max(c.align for _, c in copies)
        explicit = any(c.explicit for _, c in copies)
    else:
        lb = ub = 0
        align = 1
        explicit = False
    return TM(entries, lb, ub, align, explicit)


def typemap(spec) -> TM:
    k = spec[0]
    if k == "basic":
        s = SIZES[spec[1]]
        return TM([(0, s)], 0, s, s, False)
    if k == "contiguous":
        n, c = spec[1], typemap(spec[2])
        return _place([(i * c.extent, c) for i in range(n)])
    if k == "vector":
        n, bl, st, c = spec[1], spec[2], spec[3], typemap(spec[4])
        return _place([((i * st + j) * c.extent, c) for i in range(n) for j in range(bl)])
    if k == "hvector":
        n, bl, st, c = spec[1], spec[2], spec[3], typemap(spec[4])
        return _place([(i * st + j * c.extent, c) for i in range(n) for j in range(bl)])
    if k == "indexed":
        bls, dps, c = list(spec[1]), list(spec[2]), typemap(spec[3])
        return _place([((int(d) + j) * c.extent, c) for b, d in zip(bls, dps) for j in range(int(b))])
    if k == "hindexed":
        bls, dps, c = list(spec[1]), list(spec[2]), typemap(spec[3])
        return _place([(int(d) + j * c.extent, c) for b, d in zip(bls, dps) for j in range(int(b))])
    if k == "indexed_block":
        bl, dps, c = spec[1], list(spec[2]), typemap(spec[3])
        return _place([((int(d) + j) * c.extent, c) for d in dps for j in range(bl)])
    if k == "hindexed_block":
        bl, dps, c = spec[1], list(spec[2]), typemap(spec[3])
        return _place([(int(d) + j * c.extent, c) for d in dps for j in range(bl)])
    if k == "struct":
        bls, dps, kids = list(spec[1]), list(spec[2]), [typemap(x) for x in spec[3]]
        t = _place([(int(d) + j * c.extent, c) for b, d, c in zip(bls, dps, kids) for j in range(int(b))])
        # natural alignment padding unless a member carries explicit bounds
        if not t.explicit and t.extent > 0 and t.extent % t.align:
            t.ub += t.align - t.extent % t.align
        return t
    if k == "subarray":
        sizes, subs, starts, order, c = spec[1], spec[2], spec[3], spec[4], typemap(spec[5])
        nd = len(sizes)
        # all index tuples of the sub-box, in the order the layout lists them
        tuples = [()]
        dims = range(nd) if order == "C" else reversed(range(nd))
        for k2 in dims:
            rng_k = range(starts[k2], starts[k2] + subs[k2])
            if order == "C":
                tuples = [t + (i,) for t in tuples for i in rng_k]
            else:
                tuples = [(i,) + t for t in tuples for i in rng_k]
        if any(s == 0 for s in subs):
            tuples = []

        def lin(t):
            if order == "C":
                v = 0
                for k3 in range(nd):
                    v = v * sizes[k3] + t[k3]
                return v
            v = 0
            for k3 in reversed(range(nd)):
                v = v * sizes[k3] + t[k3]
            return v

        t = _place([(lin(tp) * c.extent, c) for tp in tuples])
        total = 1
        for s in sizes:
            total *= s
        t.lb, t.ub, t.explicit = 0, total * c.extent, True
        return t
    if k == "resized":
        lb, ext, c = spec[1], spec[2], typemap(spec[3])
        return TM(list(c.entries), lb, lb + ext, c.align, True)
    if k == "dup":
        c = typemap(spec[1])
        return TM(list(c.entries), c.lb, c.ub, c.align, c.explicit)
    raise ValueError(k)


def repeat(tm: TM, count: int) -> TM:
    """The typemap of `count` consecutive elements (element r shifted by
    r * extent), as one entry list."""
    entries = [(r * tm.extent + d, s) for r in range(count) for d, s in tm.entries]
    return TM(entries, tm.lb, tm.lb + count * tm.extent, tm.align, tm.explicit)


def segments(tm: TM):
    """Maximal runs, in map order, of entries that start where the previous ended."""
    segs = []
    for d, s in tm.entries:
        if segs and segs[-1][0] + segs[-1][1] == d:
            segs[-1][1] += s
        else:
            segs.append([d, s])
    return [tuple(x) for x in segs]


def iov_len(tm: TM, max_bytes: int):
    segs = segments(tm)
    if max_bytes == -1 or max_bytes > tm.size:
        return len(segs), tm.size
    n = acc = 0
    for _, ln in segs:
        if acc + ln > max_bytes:
            break
        acc += ln
        n += 1
    return n, acc


def iov(tm: TM, off: int, m: int):
    return segments(tm)[off:off + m]


def stream_addrs(tm: TM, count: int):
    """Byte address (relative to origin) of every packed byte, in order."""
    out = []
    for r in range(count):
        for d, s in tm.entries:
            base = r * tm.extent + d
            out.extend(range(base, base + s))
    return np.array(out, dtype=np.int64)


def pack(tm: TM, buf: np.ndarray, origin: int, count: int, off: int = 0, max_bytes: int = -1):
    addrs = stream_addrs(tm, count)
    end = len(addrs) if max_bytes < 0 else min(len(addrs), off + max_bytes)
    sel = addrs[off:end] if off < len(addrs) else addrs[:0]
    return buf[origin + sel].copy()


def unpack(tm: TM, packed: np.ndarray, buf: np.ndarray, origin: int, count: int, off: int = 0):
    addrs = stream_addrs(tm, count)
    sel = addrs[off:off + len(packed)]
    assert len(sel) == len(packed)
    buf[origin + sel] = packed


def overlaps(tm: TM, count: int) -> bool:
    addrs = stream_addrs(tm, count)
    return len(np.unique(addrs)) != len(addrs)
