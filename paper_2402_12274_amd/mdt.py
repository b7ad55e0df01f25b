"""ctypes binding of libmdt.so (C ABI in include/mdt.h).

Argument marshalling only: every step of type compilation, segment queries
and data movement runs in the native library and its gfx950 kernels.  The
functions keep the C names; ``Type`` is a small owning wrapper around a type
handle and ``build_type`` turns an input spec (see ``inputs``) into one.

Importing this module loads the library and raises ImportError when it has
not been built (``python -m paper_2402_12274_amd.build``): there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2402_12274_amd.build`")

# One HIP runtime per process: PyTorch ships its own libamdhip64 and loads it
# under a name the dynamic loader does not match against an already loaded
# system copy, so torch (when present) is imported first and libmdt then
# binds to that same runtime by soname.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_lib = C.CDLL(LIB_PATH)

# error codes (include/mdt.h)
SUCCESS, ERR_ARG, ERR_TYPE, ERR_COUNT, ERR_TRUNCATE, ERR_OVERLAP, ERR_NO_MEM, ERR_HIP, ERR_AGAIN, ERR_STATE = range(10)
ORDER_C, ORDER_FORTRAN = 0, 1
DISTRIBUTE_NONE, DISTRIBUTE_BLOCK, DISTRIBUTE_CYCLIC, DISTRIBUTE_DFLT_DARG = 0, 1, 2, -1
BASIC_CODES = {
    "BYTE": 0, "CHAR": 1, "INT8": 2, "UINT8": 3, "INT16": 4, "UINT16": 5, "INT32": 6, "UINT32": 7,
    "INT": 8, "FLOAT": 9, "INT64": 10, "UINT64": 11, "DOUBLE": 12,
}

_P = C.c_void_p
_I64 = C.c_int64
_I64P = C.POINTER(C.c_int64)
_INT = C.c_int


class Iov(C.Structure):
    _fields_ = [("iov_base", C.c_void_p), ("iov_len", C.c_int64)]


class BatchConfig(C.Structure):
    _fields_ = [("tile_chunks", C.c_int), ("wgs_per_cu", C.c_int), ("policy", C.c_int), ("use_graph", C.c_int),
                ("order", C.c_int)]


class LayoutInfo(C.Structure):
    _fields_ = [("kind", C.c_int32), ("records", C.c_int32), ("groups", C.c_int64), ("runs", C.c_int64),
                ("record_bytes", C.c_int64), ("record_stride", C.c_int64), ("pack_table", C.c_int32),
                ("unpack_table", C.c_int32), ("device_bytes", C.c_int64)]


class ServerConfig(C.Structure):
    _fields_ = [("nstreams", C.c_int), ("budget_bytes", C.c_int64), ("max_batch", C.c_int),
                ("max_inflight", C.c_int), ("arena_bytes", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("deferred", C.c_int64), ("bytes", C.c_int64), ("launches", C.c_int64),
                ("p50_us", C.c_double), ("p99_us", C.c_double), ("max_us", C.c_double),
                ("elapsed_s", C.c_double), ("inflight_bytes", C.c_int64), ("peak_inflight_bytes", C.c_int64),
                ("p50_queue_us", C.c_double), ("p99_queue_us", C.c_double), ("p50_run_us", C.c_double),
                ("p99_run_us", C.c_double), ("direct", C.c_int64)]


# generalized-request callbacks (include/mdt.h)
GREQ_QUERY_FN = C.CFUNCTYPE(_INT, _P)
GREQ_FREE_FN = C.CFUNCTYPE(_INT, _P)
GREQ_CANCEL_FN = C.CFUNCTYPE(_INT, _P, _INT)
GREQ_POLL_FN = C.CFUNCTYPE(_INT, _P)
GREQ_WAIT_FN = C.CFUNCTYPE(_INT, _INT, C.POINTER(_P), C.c_double)

_SIGS = {
    "mdt_basic": ([_INT], _P),
    "mdt_type_contiguous": ([_I64, _P, C.POINTER(_P)], _INT),
    "mdt_type_vector": ([_I64, _I64, _I64, _P, C.POINTER(_P)], _INT),
    "mdt_type_create_hvector": ([_I64, _I64, _I64, _P, C.POINTER(_P)], _INT),
    "mdt_type_indexed": ([_I64, _I64P, _I64P, _P, C.POINTER(_P)], _INT),
    "mdt_type_create_hindexed": ([_I64, _I64P, _I64P, _P, C.POINTER(_P)], _INT),
    "mdt_type_create_indexed_block": ([_I64, _I64, _I64P, _P, C.POINTER(_P)], _INT),
    "mdt_type_create_hindexed_block": ([_I64, _I64, _I64P, _P, C.POINTER(_P)], _INT),
    "mdt_type_create_struct": ([_I64, _I64P, _I64P, C.POINTER(_P), C.POINTER(_P)], _INT),
    "mdt_type_create_subarray": ([_INT, _I64P, _I64P, _I64P, _INT, _P, C.POINTER(_P)], _INT),
    "mdt_type_create_darray": ([_INT, _INT, _INT, _I64P, C.POINTER(_INT), C.POINTER(_INT), C.POINTER(_INT), _INT, _P,
                                C.POINTER(_P)], _INT),
    "mdt_type_get_envelope": ([_P, _I64P, _I64P, _I64P, C.POINTER(_INT)], _INT),
    "mdt_type_get_contents": ([_P, _I64, _I64, _I64, _I64P, _I64P, C.POINTER(_P)], _INT),
    "mdt_type_create_resized": ([_P, _I64, _I64, C.POINTER(_P)], _INT),
    "mdt_type_dup": ([_P, C.POINTER(_P)], _INT),
    "mdt_type_commit": ([C.POINTER(_P)], _INT),
    "mdt_type_free": ([C.POINTER(_P)], _INT),
    "mdt_type_size": ([_P, _I64P], _INT),
    "mdt_type_layout_info": ([_P, C.POINTER(LayoutInfo)], _INT),
    "mdt_type_get_extent": ([_P, _I64P, _I64P], _INT),
    "mdt_type_get_true_extent": ([_P, _I64P, _I64P], _INT),
    "mdt_type_iov_len": ([_P, _I64, _I64P, _I64P], _INT),
    "mdt_type_iov": ([_P, _I64, C.POINTER(Iov), _I64, _I64P], _INT),
    "mdt_type_iov_len_count": ([_P, _I64, _I64, _I64P, _I64P], _INT),
    "mdt_type_iov_count": ([_P, _I64, _I64, C.POINTER(Iov), _I64, _I64P], _INT),
    "mdt_pack": ([_P, _I64, _P, _I64, _P, _I64, _I64P], _INT),
    "mdt_unpack": ([_P, _I64, _P, _I64, _P, _I64, _I64P], _INT),
    "mdt_typed_copy": ([_P, _I64, _P, _P, _I64, _P, _I64, _I64, _I64P], _INT),
    "mdt_typed_copy_enqueue": ([_P, _I64, _P, _P, _I64, _P, _I64, _I64, _I64P, _P, C.POINTER(_P)], _INT),
    "mdt_stream_create": ([_P, C.POINTER(_P)], _INT),
    "mdt_stream_free": ([C.POINTER(_P)], _INT),
    "mdt_pack_enqueue": ([_P, _I64, _P, _I64, _P, _I64, _I64P, _P, C.POINTER(_P)], _INT),
    "mdt_unpack_enqueue": ([_P, _I64, _P, _I64, _P, _I64, _I64P, _P, C.POINTER(_P)], _INT),
    "mdt_type_iov_enqueue": ([_P, _I64, _P, _I64, _P, _I64P, _P, C.POINTER(_P)], _INT),
    "mdt_type_iov_count_enqueue": ([_P, _I64, _I64, _P, _I64, _P, _I64P, _P, C.POINTER(_P)], _INT),
    "mdt_wait": ([C.POINTER(_P)], _INT),
    "mdt_test": ([C.POINTER(_P), C.POINTER(_INT)], _INT),
    "mdt_waitall": ([_INT, C.POINTER(_P)], _INT),
    "mdt_grequest_start": ([GREQ_QUERY_FN, GREQ_FREE_FN, GREQ_CANCEL_FN, GREQ_POLL_FN, GREQ_WAIT_FN, _P,
                            C.POINTER(_P)], _INT),
    "mdt_grequest_complete": ([_P], _INT),
    "mdt_cancel": ([_P], _INT),
    "mdt_stream_progress": ([_P], _INT),
    "mdt_start_progress_thread": ([_P], _INT),
    "mdt_stop_progress_thread": ([_P], _INT),
    "mdt_request_get_status": ([_P, C.POINTER(_INT)], _INT),
    "mdt_batch_create": ([C.POINTER(_P)], _INT),
    "mdt_batch_free": ([C.POINTER(_P)], _INT),
    "mdt_batch_clear": ([_P], _INT),
    "mdt_batch_add_pack": ([_P, _P, _I64, _P, _I64, _P, _I64, _I64P], _INT),
    "mdt_batch_add_unpack": ([_P, _P, _I64, _P, _I64, _P, _I64, _I64P], _INT),
    "mdt_batch_add_copy": ([_P, _P, _I64, _P, _P, _I64, _P, _I64, _I64, _I64P], _INT),
    "mdt_batch_add_relay": ([_P, _P, _I64, _P, _P, _P, _I64, _P, _I64, _I64, _I64P], _INT),
    "mdt_batch_set_config": ([_P, C.POINTER(BatchConfig)], _INT),
    "mdt_batch_get_config": ([_P, C.POINTER(BatchConfig)], _INT),
    "mdt_batch_autotune": ([_P, _P, C.POINTER(BatchConfig)], _INT),
    "mdt_batch_autotune_set": ([_INT, C.POINTER(_P), _P, C.POINTER(BatchConfig)], _INT),
    "mdt_batch_launch": ([_P, _P, C.POINTER(_P)], _INT),
    "mdt_batch_launch_noalloc": ([_P, _P], _INT),
    "mdt_server_create": ([C.POINTER(ServerConfig), C.POINTER(_P)], _INT),
    "mdt_server_free": ([C.POINTER(_P)], _INT),
    "mdt_server_submit_pack": ([_P, _P, _I64, _P, _I64, _I64, C.POINTER(_P)], _INT),
    "mdt_server_submit_unpack": ([_P, _P, _I64, _P, _I64, _P, _I64, C.POINTER(_P)], _INT),
    "mdt_server_request_test": ([_P, _P, C.POINTER(_INT)], _INT),
    "mdt_server_request_wait": ([_P, _P], _INT),
    "mdt_server_request_result": ([_P, _P, C.POINTER(_INT), C.POINTER(_P), _I64P, C.POINTER(C.c_double)], _INT),
    "mdt_server_request_release": ([_P, C.POINTER(_P)], _INT),
    "mdt_server_progress": ([_P], _INT),
    "mdt_server_start_progress_thread": ([_P], _INT),
    "mdt_server_stop_progress_thread": ([_P], _INT),
    "mdt_server_stats_get": ([_P, C.POINTER(ServerStats)], _INT),
    "mdt_server_inject_alloc_failures": ([_P, _INT], _INT),
    "mdt_error_string": ([_INT], C.c_char_p),
    "mdt_last_hip_error": ([], _INT),
    "mdt_version": ([], _INT),
}

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name, None)
    if _f is not None:
        _f.argtypes = _args
        _f.restype = _res

SYMBOLS = tuple(_SIGS)


class MdtError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = _lib.mdt_error_string(code).decode()
        if code == ERR_HIP:
            msg += f" (hip error {_lib.mdt_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{code}]")
        self.code = code


def check(rc: int, what: str = "mdt"):
    if rc != SUCCESS:
        raise MdtError(rc, what)


def _arr(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    return a, a.ctypes.data_as(_I64P)


def lib():
    return _lib


# ---------------------------------------------------------------------------
# types


class Type:
    """Owning wrapper of an mdt_type handle."""

    def __init__(self, handle: int, owned: bool = True):
        self.handle = handle
        self.owned = owned

    def __del__(self):
        try:
            if getattr(self, "owned", False) and self.handle:
                h = _P(self.handle)
                _lib.mdt_type_free(C.byref(h))
                self.handle = None
        except Exception:  # interpreter shutdown: module globals may be gone
            pass

    @property
    def h(self):
        return _P(self.handle)

    def commit(self) -> "Type":
        h = _P(self.handle)
        check(_lib.mdt_type_commit(C.byref(h)), "commit")
        return self

    def size(self) -> int:
        v = C.c_int64()
        check(_lib.mdt_type_size(self.h, C.byref(v)), "size")
        return v.value

    def layout_info(self) -> dict:
        """Summary of the committed layout program (kind, groups, runs, record
        view and its tables, resident device bytes)."""
        v = LayoutInfo()
        check(_lib.mdt_type_layout_info(self.h, C.byref(v)), "layout_info")
        return {f: getattr(v, f) for f, _ in v._fields_}

    def extent(self):
        a, b = C.c_int64(), C.c_int64()
        check(_lib.mdt_type_get_extent(self.h, C.byref(a), C.byref(b)), "extent")
        return a.value, b.value

    def true_extent(self):
        a, b = C.c_int64(), C.c_int64()
        check(_lib.mdt_type_get_true_extent(self.h, C.byref(a), C.byref(b)), "true_extent")
        return a.value, b.value

    def iov_len(self, max_iov_bytes: int, count: int = None):
        """mdt_type_iov_len, or mdt_type_iov_len_count when count is given."""
        a, b = C.c_int64(), C.c_int64()
        if count is None:
            check(_lib.mdt_type_iov_len(self.h, max_iov_bytes, C.byref(a), C.byref(b)), "iov_len")
        else:
            check(_lib.mdt_type_iov_len_count(self.h, count, max_iov_bytes, C.byref(a), C.byref(b)), "iov_len_count")
        return a.value, b.value

    def iov(self, iov_offset: int, max_iov_len: int, count: int = None):
        """mdt_type_iov, or mdt_type_iov_count when count is given."""
        m = max(0, max_iov_len)
        buf = (Iov * max(1, m))()
        got = C.c_int64()
        if count is None:
            check(_lib.mdt_type_iov(self.h, iov_offset, buf, max_iov_len, C.byref(got)), "iov")
        else:
            check(_lib.mdt_type_iov_count(self.h, count, iov_offset, buf, max_iov_len, C.byref(got)), "iov_count")
        n = got.value
        base = np.array([(buf[i].iov_base or 0) for i in range(n)], dtype=np.uint64).view(np.int64)
        ln = np.array([buf[i].iov_len for i in range(n)], dtype=np.int64)
        return base, ln


def basic(name: str) -> Type:
    return Type(_lib.mdt_basic(BASIC_CODES[name]), owned=False)


def _new(fn, *args, what="constructor") -> Type:
    out = _P()
    check(fn(*args, C.byref(out)), what)
    return Type(out.value)


COMBINERS = ("named", "dup", "contiguous", "vector", "hvector", "indexed", "hindexed", "indexed_block",
             "hindexed_block", "struct", "subarray", "darray", "resized")


def envelope(t: Type):
    """(combiner name, number of integers, addresses, datatypes)."""
    ni, na, nt, comb = C.c_int64(), C.c_int64(), C.c_int64(), _INT()
    check(_lib.mdt_type_get_envelope(t.h, C.byref(ni), C.byref(na), C.byref(nt), C.byref(comb)), "get_envelope")
    return COMBINERS[comb.value], ni.value, na.value, nt.value


def spec_of(t: Type):
    """The constructor spec a type was built from, read back through its
    envelope and contents (recursively): build_type(spec_of(t)) rebuilds it."""
    comb, ni, na, nt = envelope(t)
    if comb == "named":
        names = {_lib.mdt_basic(code): name for name, code in BASIC_CODES.items()}
        return ("basic", names[t.h.value])
    ints = np.zeros(max(ni, 1), np.int64)
    addrs = np.zeros(max(na, 1), np.int64)
    kids = (_P * max(nt, 1))()
    check(_lib.mdt_type_get_contents(t.h, ni, na, nt, ints.ctypes.data_as(_I64P), addrs.ctypes.data_as(_I64P), kids),
          "get_contents")
    iv = [int(x) for x in ints[:ni]]
    av = [int(x) for x in addrs[:na]]
    # derived children come back as new references (freed when the wrapper
    # goes); predefined ones as themselves (freeing those is a no-op error)
    ch = [spec_of(Type(kids[i])) for i in range(nt)]
    order = {ORDER_C: "C", ORDER_FORTRAN: "F"}
    if comb == "dup":
        return ("dup", ch[0])
    if comb == "contiguous":
        return ("contiguous", iv[0], ch[0])
    if comb == "vector":
        return ("vector", iv[0], iv[1], iv[2], ch[0])
    if comb == "hvector":
        return ("hvector", iv[0], iv[1], av[0], ch[0])
    if comb == "indexed":
        n = iv[0]
        return ("indexed", iv[1:1 + n], iv[1 + n:1 + 2 * n], ch[0])
    if comb == "hindexed":
        return ("hindexed", iv[1:], av, ch[0])
    if comb == "indexed_block":
        return ("indexed_block", iv[1], iv[2:], ch[0])
    if comb == "hindexed_block":
        return ("hindexed_block", iv[1], av, ch[0])
    if comb == "struct":
        return ("struct", iv[1:], av, ch)
    if comb == "subarray":
        nd = iv[0]
        return ("subarray", iv[1:1 + nd], iv[1 + nd:1 + 2 * nd], iv[1 + 2 * nd:1 + 3 * nd], order[iv[-1]], ch[0])
    if comb == "darray":
        size, rank, nd = iv[0], iv[1], iv[2]
        g = iv[3:3 + nd]
        dist = [{DISTRIBUTE_NONE: "none", DISTRIBUTE_BLOCK: "block", DISTRIBUTE_CYCLIC: "cyclic"}[d]
                for d in iv[3 + nd:3 + 2 * nd]]
        darg = [None if a == DISTRIBUTE_DFLT_DARG else a for a in iv[3 + 2 * nd:3 + 3 * nd]]
        return ("darray", size, rank, g, dist, darg, iv[3 + 3 * nd:3 + 4 * nd], order[iv[-1]], ch[0])
    if comb == "resized":
        return ("resized", av[0], av[1], ch[0])
    raise ValueError(comb)


def build_type(spec, commit: bool = True) -> Type:
    """Build (and commit) a type from an input spec (nested constructor tuples)."""
    t = _build(spec)
    if commit:
        t.commit()
    return t


def _build(spec) -> Type:
    k = spec[0]
    if k == "basic":
        return basic(spec[1])
    if k == "contiguous":
        c = _build(spec[2])
        return _new(_lib.mdt_type_contiguous, spec[1], c.h, what=k)
    if k == "vector":
        _, n, bl, st, child = spec
        c = _build(child)
        return _new(_lib.mdt_type_vector, n, bl, st, c.h, what=k)
    if k == "hvector":
        _, n, bl, st, child = spec
        c = _build(child)
        return _new(_lib.mdt_type_create_hvector, n, bl, st, c.h, what=k)
    if k in ("indexed", "hindexed"):
        _, bls, disps, child = spec
        c = _build(child)
        b, bp = _arr(bls)
        d, dp = _arr(disps)
        f = _lib.mdt_type_indexed if k == "indexed" else _lib.mdt_type_create_hindexed
        return _new(f, b.size, bp, dp, c.h, what=k)
    if k in ("indexed_block", "hindexed_block"):
        _, bl, disps, child = spec
        c = _build(child)
        d, dp = _arr(disps)
        f = _lib.mdt_type_create_indexed_block if k == "indexed_block" else _lib.mdt_type_create_hindexed_block
        return _new(f, d.size, bl, dp, c.h, what=k)
    if k == "struct":
        _, bls, disps, children = spec
        kids = [_build(x) for x in children]
        b, bp = _arr(bls)
        d, dp = _arr(disps)
        arr = (_P * max(1, len(kids)))(*[x.handle for x in kids])
        return _new(_lib.mdt_type_create_struct, b.size, bp, dp, arr, what=k)
    if k == "subarray":
        _, sizes, subs, starts, order, child = spec
        c = _build(child)
        s, sp = _arr(sizes)
        u, up = _arr(subs)
        t, tp = _arr(starts)
        o = {"C": ORDER_C, "F": ORDER_FORTRAN}.get(order, 7)
        return _new(_lib.mdt_type_create_subarray, s.size, sp, up, tp, o, c.h, what=k)
    if k == "darray":
        # ("darray", size, rank, gsizes, distribs ("none"|"block"|"cyclic"),
        #  dargs (int, or None for the default), psizes, order, child)
        _, size, rank, gsizes, distribs, dargs, psizes, order, child = spec
        c = _build(child)
        g, gp = _arr(gsizes)
        nd = g.size
        ints = lambda v: (_INT * max(1, nd))(*v)
        dist = ints([{"none": DISTRIBUTE_NONE, "block": DISTRIBUTE_BLOCK, "cyclic": DISTRIBUTE_CYCLIC}.get(d, 9)
                     for d in distribs])
        darg = ints([DISTRIBUTE_DFLT_DARG if a is None else a for a in dargs])
        o = {"C": ORDER_C, "F": ORDER_FORTRAN}.get(order, 7)
        return _new(_lib.mdt_type_create_darray, size, rank, nd, gp, dist, darg, ints(psizes), o, c.h, what=k)
    if k == "resized":
        _, lb, ext, child = spec
        c = _build(child)
        return _new(_lib.mdt_type_create_resized, c.h, lb, ext, what=k)
    if k == "dup":
        c = _build(spec[1])
        return _new(_lib.mdt_type_dup, c.h, what=k)
    raise ValueError(f"unknown constructor {k!r}")


# ---------------------------------------------------------------------------
# data movement (device pointers as ints)


def mdt_pack(inbuf: int, incount: int, t: Type, inoffset: int, outbuf: int, max_pack_bytes: int = -1) -> int:
    n = C.c_int64()
    check(_lib.mdt_pack(_P(inbuf), incount, t.h, inoffset, _P(outbuf), max_pack_bytes, C.byref(n)), "mdt_pack")
    return n.value


def mdt_unpack(inbuf: int, insize: int, outbuf: int, outcount: int, t: Type, outoffset: int = 0) -> int:
    n = C.c_int64()
    check(_lib.mdt_unpack(_P(inbuf), insize, _P(outbuf), outcount, t.h, outoffset, C.byref(n)), "mdt_unpack")
    return n.value


def mdt_typed_copy(src: int, srccount: int, srctype: Type, dst: int, dstcount: int, dsttype: Type, offset: int = 0,
                   max_bytes: int = -1) -> int:
    """Stream bytes [offset, offset + n) of (srccount x srctype) at src to the
    same positions of (dstcount x dsttype) at dst, in one pass."""
    n = C.c_int64()
    check(_lib.mdt_typed_copy(_P(src), srccount, srctype.h, _P(dst), dstcount, dsttype.h, offset, max_bytes,
                              C.byref(n)), "mdt_typed_copy")
    return n.value


class Stream:
    """mdt_stream wrapping a HIP stream handle (int; 0 = null stream)."""

    def __init__(self, hip_stream: int = 0):
        self.handle = _P()
        check(_lib.mdt_stream_create(_P(hip_stream), C.byref(self.handle)), "stream_create")

    def __del__(self):
        try:
            if getattr(self, "handle", None) and self.handle.value:
                _lib.mdt_stream_free(C.byref(self.handle))
        except Exception:
            pass

    @property
    def h(self):
        return self.handle


class Request:
    def __init__(self):
        self.handle = _P()

    def wait(self):
        check(_lib.mdt_wait(C.byref(self.handle)), "wait")

    def test(self) -> bool:
        f = C.c_int()
        check(_lib.mdt_test(C.byref(self.handle), C.byref(f)), "test")
        return bool(f.value)

    def status(self) -> bool:
        """mdt_request_get_status: complete as far as progress has seen (no
        progress, the request is not freed)."""
        f = C.c_int()
        check(_lib.mdt_request_get_status(self.handle, C.byref(f)), "request_get_status")
        return bool(f.value)


def _stream_handle(stream):
    return stream.h if stream is not None else None


def stream_progress(stream=None):
    """mdt_stream_progress (None: general progress)."""
    check(_lib.mdt_stream_progress(_stream_handle(stream)), "stream_progress")


def start_progress_thread(stream=None):
    check(_lib.mdt_start_progress_thread(_stream_handle(stream)), "start_progress_thread")


def stop_progress_thread(stream=None):
    check(_lib.mdt_stop_progress_thread(_stream_handle(stream)), "stop_progress_thread")


def waitall(reqs):
    """mdt_waitall over Request objects (None entries allowed)."""
    arr = (_P * len(reqs))(*[r.handle.value if r is not None else None for r in reqs])
    rc = _lib.mdt_waitall(len(reqs), arr)
    for r, h in zip(reqs, arr):
        if r is not None:
            r.handle = _P(h)
    check(rc, "waitall")


# live generalized requests by key (their extra_state), so the callbacks
# and the Python state outlive the call that started them
_GREQS = {}
_GREQ_NEXT = [1]
# one C wrapper per Python wait callable: requests that share the callable
# share the C function pointer, so the library groups them into one call.
# Wrappers live as long as the process (pass the same function object, not a
# fresh lambda or bound method per request, to share one and to group).
_WAIT_WRAPPERS = {}


def _wait_wrapper(wait):
    w = _WAIT_WRAPPERS.get(wait)
    if w is None:
        w = GREQ_WAIT_FN(lambda n, st, t: int(wait([_GREQS[st[i]] for i in range(n)], t) or 0))
        _WAIT_WRAPPERS[wait] = w
    return w


class GRequest(Request):
    """Generalized request (mdt_grequest_start) driven by Python callables.

    poll(g) checks the task and calls g.complete() once it has finished;
    wait(list_of_g, timeout) blocks on several of them at once; query(g),
    free(g) and cancel(g, complete) follow include/mdt.h.  Each callable
    returns None or 0 for success, or an int error code."""

    def __init__(self, poll=None, wait=None, query=None, free=None, cancel=None, state=None):
        super().__init__()
        self.state = state
        self.key = _GREQ_NEXT[0]
        _GREQ_NEXT[0] += 1
        rc = lambda v: int(v or 0)
        me = self

        def _free(_):
            try:
                return rc(free(me)) if free else 0
            finally:
                _GREQS.pop(me.key, None)

        # an absent callback is a NULL function pointer (the type called
        # with no argument)
        cbs = (
            GREQ_QUERY_FN(lambda _: rc(query(me))) if query else GREQ_QUERY_FN(),
            GREQ_FREE_FN(_free),
            GREQ_CANCEL_FN(lambda _, c: rc(cancel(me, bool(c)))) if cancel else GREQ_CANCEL_FN(),
            GREQ_POLL_FN(lambda _: rc(poll(me))) if poll else GREQ_POLL_FN(),
            _wait_wrapper(wait) if wait else GREQ_WAIT_FN(),
        )
        self._cbs = cbs
        _GREQS[self.key] = self
        try:
            check(_lib.mdt_grequest_start(*cbs, _P(self.key), C.byref(self.handle)), "grequest_start")
        except Exception:
            _GREQS.pop(self.key, None)
            raise

    def complete(self):
        check(_lib.mdt_grequest_complete(self.handle), "grequest_complete")

    def cancel(self):
        check(_lib.mdt_cancel(self.handle), "cancel")


def mdt_pack_enqueue(inbuf: int, incount: int, t: Type, inoffset: int, outbuf: int, max_pack_bytes: int,
                     stream: Stream, want_request: bool = False):
    n = C.c_int64()
    req = Request() if want_request else None
    check(_lib.mdt_pack_enqueue(_P(inbuf), incount, t.h, inoffset, _P(outbuf), max_pack_bytes, C.byref(n), stream.h,
                                C.byref(req.handle) if req else None), "mdt_pack_enqueue")
    return n.value, req


def mdt_typed_copy_enqueue(src: int, srccount: int, srctype: Type, dst: int, dstcount: int, dsttype: Type,
                           offset: int, max_bytes: int, stream: Stream, want_request: bool = False):
    n = C.c_int64()
    req = Request() if want_request else None
    check(_lib.mdt_typed_copy_enqueue(_P(src), srccount, srctype.h, _P(dst), dstcount, dsttype.h, offset, max_bytes,
                                      C.byref(n), stream.h, C.byref(req.handle) if req else None),
          "mdt_typed_copy_enqueue")
    return n.value, req


def mdt_unpack_enqueue(inbuf: int, insize: int, outbuf: int, outcount: int, t: Type, outoffset: int,
                       stream: Stream, want_request: bool = False):
    n = C.c_int64()
    req = Request() if want_request else None
    check(_lib.mdt_unpack_enqueue(_P(inbuf), insize, _P(outbuf), outcount, t.h, outoffset, C.byref(n), stream.h,
                                  C.byref(req.handle) if req else None), "mdt_unpack_enqueue")
    return n.value, req


def mdt_type_iov_enqueue(t: Type, iov_offset: int, dev_iov: int, max_iov_len: int, base: int, stream: Stream,
                         want_request: bool = False):
    n = C.c_int64()
    req = Request() if want_request else None
    check(_lib.mdt_type_iov_enqueue(t.h, iov_offset, _P(dev_iov), max_iov_len, _P(base), C.byref(n), stream.h,
                                    C.byref(req.handle) if req else None), "mdt_type_iov_enqueue")
    return n.value, req


def mdt_type_iov_count_enqueue(t: Type, count: int, iov_offset: int, dev_iov: int, max_iov_len: int, base: int,
                               stream: Stream, want_request: bool = False):
    n = C.c_int64()
    req = Request() if want_request else None
    check(_lib.mdt_type_iov_count_enqueue(t.h, count, iov_offset, _P(dev_iov), max_iov_len, _P(base), C.byref(n),
                                          stream.h, C.byref(req.handle) if req else None),
          "mdt_type_iov_count_enqueue")
    return n.value, req


# ---------------------------------------------------------------------------
# batches


class Batch:
    """mdt_batch: many requests in one persistent (graph-captured) launch."""

    def __init__(self):
        self.handle = _P()
        check(_lib.mdt_batch_create(C.byref(self.handle)), "batch_create")
        self._keep = []

    def __del__(self):
        try:
            if getattr(self, "handle", None) and self.handle.value:
                _lib.mdt_batch_free(C.byref(self.handle))
        except Exception:
            pass

    def clear(self):
        check(_lib.mdt_batch_clear(self.handle), "batch_clear")
        self._keep = []

    def add_pack(self, inbuf: int, incount: int, t: Type, inoffset: int, outbuf: int, max_pack_bytes: int = -1):
        n = C.c_int64()
        check(_lib.mdt_batch_add_pack(self.handle, _P(inbuf), incount, t.h, inoffset, _P(outbuf), max_pack_bytes,
                                      C.byref(n)), "batch_add_pack")
        self._keep.append(t)
        return n.value

    def add_unpack(self, inbuf: int, insize: int, outbuf: int, outcount: int, t: Type, outoffset: int = 0):
        n = C.c_int64()
        check(_lib.mdt_batch_add_unpack(self.handle, _P(inbuf), insize, _P(outbuf), outcount, t.h, outoffset,
                                        C.byref(n)), "batch_add_unpack")
        self._keep.append(t)
        return n.value

    def add_copy(self, src: int, srccount: int, srctype: Type, dst: int, dstcount: int, dsttype: Type,
                 offset: int = 0, max_bytes: int = -1) -> int:
        n = C.c_int64()
        check(_lib.mdt_batch_add_copy(self.handle, _P(src), srccount, srctype.h, _P(dst), dstcount, dsttype.h,
                                      offset, max_bytes, C.byref(n)), "batch_add_copy")
        self._keep.extend((srctype, dsttype))
        return n.value

    def add_relay(self, src: int, srccount: int, srctype: Type, packed: int, dst: int, dstcount: int, dsttype: Type,
                  offset: int = 0, max_bytes: int = -1) -> int:
        n = C.c_int64()
        check(_lib.mdt_batch_add_relay(self.handle, _P(src), srccount, srctype.h, _P(packed), _P(dst), dstcount,
                                       dsttype.h, offset, max_bytes, C.byref(n)), "batch_add_relay")
        self._keep.extend((srctype, dsttype))
        return n.value

    def set_config(self, cfg: BatchConfig):
        check(_lib.mdt_batch_set_config(self.handle, C.byref(cfg)), "batch_set_config")

    def get_config(self) -> BatchConfig:
        cfg = BatchConfig()
        check(_lib.mdt_batch_get_config(self.handle, C.byref(cfg)), "batch_get_config")
        return cfg

    def autotune(self, stream: Stream) -> BatchConfig:
        cfg = BatchConfig()
        check(_lib.mdt_batch_autotune(self.handle, stream.h, C.byref(cfg)), "batch_autotune")
        return cfg

    def launch(self, stream: Stream, want_request: bool = False):
        req = Request() if want_request else None
        check(_lib.mdt_batch_launch(self.handle, stream.h, C.byref(req.handle) if req else None), "batch_launch")
        return req


    def launch_noalloc(self, stream: Stream):
        """mdt_batch_launch_noalloc: the launch through the library's fixed
        device array (no allocation)."""
        check(_lib.mdt_batch_launch_noalloc(self.handle, stream.h), "batch_launch_noalloc")


def autotune_set(batches, stream: Stream) -> BatchConfig:
    """mdt_batch_autotune_set: one configuration for batches of one shape,
    timed over all of them in turn."""
    arr = (_P * len(batches))(*[b.handle.value for b in batches])
    cfg = BatchConfig()
    check(_lib.mdt_batch_autotune_set(len(batches), arr, stream.h, C.byref(cfg)), "batch_autotune_set")
    return cfg


def config_dict(cfg: BatchConfig) -> dict:
    return {f: getattr(cfg, f) for f, _ in cfg._fields_}


# ---------------------------------------------------------------------------
# serving


class Server:
    """mdt_server: continuous batching of pack/unpack requests."""

    def __init__(self, nstreams=8, budget_bytes=32 << 30, max_batch=256, max_inflight=2, arena_bytes=0):
        cfg = ServerConfig(nstreams, budget_bytes, max_batch, max_inflight, arena_bytes)
        self.handle = _P()
        check(_lib.mdt_server_create(C.byref(cfg), C.byref(self.handle)), "server_create")

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            check(_lib.mdt_server_free(C.byref(self.handle)), "server_free")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit_pack(self, inbuf: int, incount: int, t: Type, inoffset: int = 0, max_pack_bytes: int = -1) -> int:
        r = _P()
        check(_lib.mdt_server_submit_pack(self.handle, _P(inbuf), incount, t.h, inoffset, max_pack_bytes,
                                          C.byref(r)), "server_submit_pack")
        return r.value

    def submit_unpack(self, inbuf: int, insize: int, outbuf: int, outcount: int, t: Type, outoffset: int = 0) -> int:
        r = _P()
        check(_lib.mdt_server_submit_unpack(self.handle, _P(inbuf), insize, _P(outbuf), outcount, t.h, outoffset,
                                            C.byref(r)), "server_submit_unpack")
        return r.value

    def test(self, req: int) -> bool:
        f = C.c_int()
        check(_lib.mdt_server_request_test(self.handle, _P(req), C.byref(f)), "server_request_test")
        return bool(f.value)

    def wait(self, req: int):
        check(_lib.mdt_server_request_wait(self.handle, _P(req)), "server_request_wait")

    def result(self, req: int):
        st, pk, nb, lat = C.c_int(), _P(), C.c_int64(), C.c_double()
        check(_lib.mdt_server_request_result(self.handle, _P(req), C.byref(st), C.byref(pk), C.byref(nb),
                                             C.byref(lat)), "server_request_result")
        return st.value, (pk.value or 0), nb.value, lat.value

    def release(self, req: int):
        r = _P(req)
        check(_lib.mdt_server_request_release(self.handle, C.byref(r)), "server_request_release")

    def progress(self):
        check(_lib.mdt_server_progress(self.handle), "server_progress")

    def start(self):
        check(_lib.mdt_server_start_progress_thread(self.handle), "start_progress_thread")

    def stop(self):
        check(_lib.mdt_server_stop_progress_thread(self.handle), "stop_progress_thread")

    def stats(self) -> dict:
        s = ServerStats()
        check(_lib.mdt_server_stats_get(self.handle, C.byref(s)), "server_stats")
        return {f: getattr(s, f) for f, _ in s._fields_}

    def inject_alloc_failures(self, n: int):
        check(_lib.mdt_server_inject_alloc_failures(self.handle, n), "inject")
