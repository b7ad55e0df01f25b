"""ctypes wrapper around ``oracle.c`` -- TEST INFRASTRUCTURE ONLY.

The oracle is the plain, slow definition of the datatype extension
(Derived Datatypes section: segment queries by byte budget and by index,
MPIX_Iov as {base, len}) and of the byte-stream pack/unpack of a count of
typemaps, including ranges that start at a byte offset and stop at a byte
budget (General Progress, Background: pipelined chunks).  It is used to
produce expected values for tests and the CPU baseline of the benchmark,
and never by the product path.

Types are described by a *spec*: nested tuples naming one constructor each
(see ``paper_2402_12274_amd.inputs`` for the format).  ``build_type`` turns a
spec into an oracle type by calling the oracle's own constructors.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Sizes of the predefined (basic) types; a basic type's alignment is its size.
_BASIC_SIZES = {
    "BYTE": 1, "CHAR": 1, "INT8": 1, "UINT8": 1,
    "INT16": 2, "UINT16": 2,
    "INT32": 4, "UINT32": 4, "INT": 4, "FLOAT": 4,
    "INT64": 8, "UINT64": 8, "DOUBLE": 8,
}

ERR_ARG, ERR_OVERLAP, ERR_TRUNCATE, ERR_NOMEM = 1, 2, 3, 4


class OracleError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__(f"oracle error {code} {what}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-Wall",
            "-shared", "-fPIC", "-pthread", "-o", tmp, _SRC,
        ])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_P = C.c_void_p
_I64 = C.c_int64
_I64P = C.POINTER(C.c_int64)


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = C.CDLL(_LIB)
    errp = C.POINTER(C.c_int)
    sigs = {
        "orc_basic": ([_I64, errp], _P),
        "orc_contiguous": ([_I64, _P, errp], _P),
        "orc_vector": ([_I64, _I64, _I64, _P, errp], _P),
        "orc_hvector": ([_I64, _I64, _I64, _P, errp], _P),
        "orc_indexed": ([_I64, _I64P, _I64P, _P, errp], _P),
        "orc_hindexed": ([_I64, _I64P, _I64P, _P, errp], _P),
        "orc_indexed_block": ([_I64, _I64, _I64P, _P, errp], _P),
        "orc_hindexed_block": ([_I64, _I64, _I64P, _P, errp], _P),
        "orc_struct": ([_I64, _I64P, _I64P, C.POINTER(_P), errp], _P),
        "orc_subarray": ([C.c_int, _I64P, _I64P, _I64P, C.c_int, _P, errp], _P),
        "orc_darray": ([C.c_int, C.c_int, C.c_int, _I64P, C.POINTER(C.c_int), C.POINTER(C.c_int),
                        C.POINTER(C.c_int), C.c_int, _P, errp], _P),
        "orc_resized": ([_P, _I64, _I64, errp], _P),
        "orc_dup": ([_P, errp], _P),
        "orc_release": ([_P], None),
        "orc_attrs": ([_P, _I64P], C.c_int),
        "orc_num_segments": ([_P, _I64P], C.c_int),
        "orc_iov_len": ([_P, _I64, _I64P, _I64P], C.c_int),
        "orc_iov": ([_P, _I64, _I64P, _I64P, _I64, _I64P], C.c_int),
        "orc_num_segments_count": ([_P, _I64, _I64P], C.c_int),
        "orc_iov_len_count": ([_P, _I64, _I64, _I64P, _I64P], C.c_int),
        "orc_iov_count": ([_P, _I64, _I64, _I64P, _I64P, _I64, _I64P], C.c_int),
        "orc_pack": ([_P, _I64, _P, _I64, _P, _I64, _I64P], C.c_int),
        "orc_pack_mt": ([_P, _I64, _P, _I64, _P, _I64, _I64P, C.c_int], C.c_int),
        "orc_unpack": ([_P, _I64, _P, _I64, _P, _I64, _I64P], C.c_int),
    }
    for name, (args, res) in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _arr(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    return a, a.ctypes.data_as(_I64P)


class OType:
    """An oracle type (owns one reference)."""

    def __init__(self, ptr, keep=()):
        self.ptr = ptr
        self._keep = keep

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.orc_release(self.ptr)
            self.ptr = None

    # -- attributes ---------------------------------------------------
    def attrs(self) -> dict:
        out = (C.c_int64 * 8)()
        load().orc_attrs(self.ptr, out)
        size, lb, ub, tlb, tub, align, expl, nent = list(out)
        return dict(size=size, lb=lb, ub=ub, extent=ub - lb, true_lb=tlb, true_ub=tub,
                    true_extent=tub - tlb, align=align, explicit=bool(expl), entries=nent)

    # -- segment queries (count consecutive elements; 1 = the type alone) --
    def num_segments(self, count: int = 1) -> int:
        n = C.c_int64()
        _check(load().orc_num_segments_count(self.ptr, count, C.byref(n)))
        return n.value

    def iov_len(self, max_iov_bytes: int, count: int = 1):
        a, b = C.c_int64(), C.c_int64()
        _check(load().orc_iov_len_count(self.ptr, count, max_iov_bytes, C.byref(a), C.byref(b)))
        return a.value, b.value

    def iov(self, iov_offset: int, max_iov_len: int, count: int = 1):
        m = max(0, max_iov_len)
        base = np.zeros(max(m, 1), np.int64)
        ln = np.zeros(max(m, 1), np.int64)
        got = C.c_int64()
        _check(load().orc_iov_count(self.ptr, count, iov_offset, base.ctypes.data_as(_I64P),
                                    ln.ctypes.data_as(_I64P), max_iov_len, C.byref(got)))
        return base[: got.value].copy(), ln[: got.value].copy()

    # -- pack / unpack --------------------------------------------------
    def pack(self, buf: np.ndarray, origin: int, count: int, inoffset: int = 0, max_bytes: int = -1,
             nthreads: int = 1) -> np.ndarray:
        """Pack from ``buf`` whose byte ``origin`` is displacement 0."""
        assert buf.dtype == np.uint8 and buf.flags.c_contiguous
        lib = load()
        total = count * self.attrs()["size"]
        n = max(0, total - inoffset)
        if max_bytes >= 0:
            n = min(n, max_bytes)
        out = np.zeros(max(n, 1), np.uint8)
        got = C.c_int64()
        org = buf.ctypes.data + origin
        if nthreads > 1:
            rc = lib.orc_pack_mt(org, count, self.ptr, inoffset, out.ctypes.data, max_bytes, C.byref(got),
                                 nthreads)
        else:
            rc = lib.orc_pack(org, count, self.ptr, inoffset, out.ctypes.data, max_bytes, C.byref(got))
        _check(rc)
        assert got.value == n
        return out[:n]

    def unpack(self, packed: np.ndarray, buf: np.ndarray, origin: int, count: int, outoffset: int = 0) -> int:
        """Unpack ``packed`` into ``buf`` (in place) whose byte ``origin`` is displacement 0."""
        assert buf.dtype == np.uint8 and buf.flags.c_contiguous
        packed = np.ascontiguousarray(packed, dtype=np.uint8)
        got = C.c_int64()
        rc = load().orc_unpack(packed.ctypes.data, packed.size, buf.ctypes.data + origin, count, self.ptr,
                               outoffset, C.byref(got))
        _check(rc)
        return got.value


def _check(rc):
    if rc != 0:
        raise OracleError(rc)


def _mk(ptr, err, keep=()):
    if not ptr:
        raise OracleError(err.value)
    return OType(ptr, keep)


def build_type(spec) -> OType:
    """Build an oracle type from a spec (nested constructor tuples)."""
    lib = load()
    err = C.c_int()
    ep = C.byref(err)
    kind = spec[0]
    if kind == "basic":
        return _mk(lib.orc_basic(_BASIC_SIZES[spec[1]], ep), err)
    if kind == "contiguous":
        c = build_type(spec[2])
        return _mk(lib.orc_contiguous(spec[1], c.ptr, ep), err)
    if kind in ("vector", "hvector"):
        _, n, bl, stride, child = spec
        c = build_type(child)
        f = lib.orc_vector if kind == "vector" else lib.orc_hvector
        return _mk(f(n, bl, stride, c.ptr, ep), err)
    if kind in ("indexed", "hindexed"):
        _, bls, disps, child = spec
        c = build_type(child)
        b, bp = _arr(bls)
        d, dp = _arr(disps)
        assert b.size == d.size
        f = lib.orc_indexed if kind == "indexed" else lib.orc_hindexed
        return _mk(f(b.size, bp, dp, c.ptr, ep), err)
    if kind in ("indexed_block", "hindexed_block"):
        _, bl, disps, child = spec
        c = build_type(child)
        d, dp = _arr(disps)
        f = lib.orc_indexed_block if kind == "indexed_block" else lib.orc_hindexed_block
        return _mk(f(d.size, bl, dp, c.ptr, ep), err)
    if kind == "struct":
        _, bls, disps, children = spec
        kids = [build_type(k) for k in children]
        b, bp = _arr(bls)
        d, dp = _arr(disps)
        assert b.size == d.size == len(kids)
        arr = (_P * max(1, len(kids)))(*[k.ptr for k in kids])
        return _mk(lib.orc_struct(b.size, bp, dp, arr, ep), err)
    if kind == "subarray":
        _, sizes, subs, starts, order, child = spec
        c = build_type(child)
        s, sp = _arr(sizes)
        u, up = _arr(subs)
        t, tp = _arr(starts)
        o = {"C": 0, "F": 1}.get(order, 7)
        return _mk(lib.orc_subarray(s.size, sp, up, tp, o, c.ptr, ep), err)
    if kind == "darray":
        # ("darray", size, rank, gsizes, distribs ("none"|"block"|"cyclic"),
        #  dargs (int, or None for the default), psizes, order, child)
        _, size, rank, gsizes, distribs, dargs, psizes, order, child = spec
        c = build_type(child)
        g, gp = _arr(gsizes)
        nd = g.size
        ints = lambda v: (C.c_int * max(1, nd))(*v)
        dist = ints([{"none": 0, "block": 1, "cyclic": 2}.get(d, 9) for d in distribs])
        darg = ints([-1 if a is None else a for a in dargs])
        ps = ints(psizes)
        o = {"C": 0, "F": 1}.get(order, 7)
        return _mk(lib.orc_darray(size, rank, nd, gp, dist, darg, ps, o, c.ptr, ep), err)
    if kind == "resized":
        _, lb, extent, child = spec
        c = build_type(child)
        return _mk(lib.orc_resized(c.ptr, lb, extent, ep), err)
    if kind == "dup":
        c = build_type(spec[1])
        return _mk(lib.orc_dup(c.ptr, ep), err)
    raise ValueError(f"unknown constructor {kind!r}")
