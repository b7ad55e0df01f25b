"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only *describes* inputs: type specs (which constructor, which
arguments) and seeded random bytes.  It holds none of the method's
arithmetic (no typemap walk, no sizes or extents, no packing), so both the
product path and the oracle can take their inputs from here without sharing
any of the computation under test.

Type spec format (one constructor per tuple, mirroring the MPI constructors
that the Derived Datatypes section builds on):

    ("basic", NAME)                                  NAME in BASIC_NAMES
    ("contiguous", n, child)
    ("vector", n, blocklength, stride, child)        stride in child extents
    ("hvector", n, blocklength, stride_bytes, child)
    ("indexed", blocklengths, displacements, child)  displacements in extents
    ("hindexed", blocklengths, displacements_bytes, child)
    ("indexed_block", blocklength, displacements, child)
    ("hindexed_block", blocklength, displacements_bytes, child)
    ("struct", blocklengths, displacements_bytes, children)
    ("subarray", sizes, subsizes, starts, "C" | "F", child)
    ("resized", lb, extent, child)
    ("dup", child)

Seeds: every generator takes an explicit seed; the default is 20240219.
"""
from __future__ import annotations

import numpy as np

DEFAULT_SEED = 20240219

BASIC_NAMES = ("BYTE", "CHAR", "INT8", "UINT8", "INT16", "UINT16", "INT32", "UINT32", "INT", "FLOAT",
               "INT64", "UINT64", "DOUBLE")

DOUBLE = ("basic", "DOUBLE")
BYTE = ("basic", "BYTE")


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_bytes(nbytes: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    """``nbytes`` seeded uniform random bytes (PCG64 64-bit words)."""
    nwords = (nbytes + 7) // 8
    words = rng(seed).integers(0, np.iinfo(np.uint64).max, size=nwords, dtype=np.uint64, endpoint=True)
    return words.view(np.uint8)[:nbytes].copy() if nwords * 8 != nbytes else words.view(np.uint8)


# ---------------------------------------------------------------------------
# small case: one vector of float64

def vector_small():
    """vector(1024, 1, 2, DOUBLE): 8 KiB packed from a 16 KiB source."""
    return ("vector", 1024, 1, 2, DOUBLE)


# ---------------------------------------------------------------------------
# 3-D halo faces of a float64 N^3 array (C order)

def halo_face(n: int, w: int, dim: int, side: str):
    """Interior face of ghost width ``w`` on dimension ``dim`` (0 slowest,
    2 fastest) of an ``n^3`` float64 array in C order.  The face spans the
    interior [w, n-w) in the other two dimensions and [w, 2w) (``lo``) or
    [n-2w, n-w) (``hi``) in ``dim``."""
    sub = [n - 2 * w] * 3
    st = [w] * 3
    sub[dim] = w
    st[dim] = w if side == "lo" else n - 2 * w
    return ("subarray", [n, n, n], sub, st, "C", DOUBLE)


def halo_faces(n: int = 512, widths=(1, 4)):
    """All 6 faces for each ghost width: list of (label, spec)."""
    out = []
    for w in widths:
        for dim in (0, 1, 2):
            for side in ("lo", "hi"):
                out.append((f"w{w}-d{dim}-{side}", halo_face(n, w, dim, side)))
    return out


# ---------------------------------------------------------------------------
# irregular layouts

def hindexed_blocks(nblocks: int = 1_000_000, span: int = 1 << 31, mean: float = 24.0, maxlen: int = 256,
                    seed: int = DEFAULT_SEED, permute: bool = True):
    """Block lengths ~ geometric(1/mean) on {1, 2, ...} clipped to [1, maxlen];
    non-overlapping byte displacements inside ``[0, span)``: the free bytes
    are split by sorted uniform cut points, blocks are laid out in address
    order, then (``permute``) the block order is shuffled so that map order
    differs from address order.  Returns (lengths, displacements) int64."""
    g = rng(seed)
    lens = np.minimum(g.geometric(1.0 / mean, size=nblocks), maxlen).astype(np.int64)
    free = span - int(lens.sum())
    if free < 0:
        raise ValueError("blocks do not fit in span")
    cuts = np.sort(g.integers(0, free + 1, size=nblocks, dtype=np.int64))
    before = np.zeros(nblocks, np.int64)
    if nblocks > 1:
        before[1:] = np.cumsum(lens)[:-1]
    disps = cuts + before
    if permute:
        perm = g.permutation(nblocks)
        lens, disps = lens[perm], disps[perm]
    return lens, disps


def hindexed_type(lens, disps):
    return ("hindexed", lens, disps, BYTE)


def particle_struct():
    """struct {int32; float64[3]; char[5]} at natural offsets 0, 8, 32."""
    return ("struct", [1, 3, 5], [0, 8, 32], [("basic", "INT32"), DOUBLE, ("basic", "CHAR")])


# ---------------------------------------------------------------------------
# batching mix

def batch_mix(nreq: int = 4096, seed: int = DEFAULT_SEED, lo: int = 64, hi: int = 16 << 20,
              n_face: int = 512, vec_count: int = 1 << 21):
    """Request descriptions for the batched-launch workload: packed sizes
    log-uniform in [lo, hi]; type drawn uniformly from {vector(vec_count, 1,
    s, DOUBLE) with s ~ U{2..64}, a halo face of an n_face^3 array, the
    hindexed layout}.  Returns a list of dicts with keys kind, spec_key,
    target (requested packed bytes)."""
    g = rng(seed)
    sizes = np.exp(g.uniform(np.log(lo), np.log(hi), size=nreq)).astype(np.int64)
    kinds = g.integers(0, 3, size=nreq)
    strides = g.integers(2, 65, size=nreq)
    faces = halo_faces(n_face)
    face_idx = g.integers(0, len(faces), size=nreq)
    reqs = []
    for i in range(nreq):
        k = int(kinds[i])
        if k == 0:
            reqs.append(dict(kind="vector", spec_key=("vector", int(strides[i])), target=int(sizes[i]),
                             spec=("vector", vec_count, 1, int(strides[i]), DOUBLE)))
        elif k == 1:
            label, spec = faces[int(face_idx[i])]
            reqs.append(dict(kind="face", spec_key=("face", label), target=int(sizes[i]), spec=spec))
        else:
            reqs.append(dict(kind="hindexed", spec_key=("hindexed",), target=int(sizes[i]), spec=None))
    return reqs


# ---------------------------------------------------------------------------
# serving trace


def serving_types(seed: int = DEFAULT_SEED, ntypes: int = 500):
    """Resident types of the serving workload: (family, spec) pairs drawn from
    strided float64 vectors, halo faces of 128^3..512^3 arrays, hindexed
    layouts with 4k..64k blocks inside 256 MiB, and particle-like records."""
    g = rng(seed)
    out = []
    fams = ["vector", "face", "hindexed", "struct"]
    for i in range(ntypes):
        fam = fams[i % 4]
        if fam == "vector":
            n = int(2 ** g.integers(12, 17))
            out.append((fam, ("vector", n, 1, int(g.integers(2, 65)), DOUBLE)))
        elif fam == "face":
            n = int(g.choice([128, 192, 256, 384, 512]))
            w = int(g.integers(1, 5))
            out.append((fam, halo_face(n, w, int(g.integers(0, 3)), "lo" if g.random() < 0.5 else "hi")))
        elif fam == "hindexed":
            nb = int(g.integers(4096, 65537))
            lens, disps = hindexed_blocks(nblocks=nb, span=1 << 28, seed=int(g.integers(0, 1 << 30)))
            out.append((fam, hindexed_type(lens, disps)))
        else:
            k = int(g.integers(1, 6))
            out.append((fam, ("struct", [1, k, 5], [0, 8, 8 + 8 * k], [("basic", "INT32"), DOUBLE, ("basic", "CHAR")])))
    return out


def serving_trace(rate: float, duration_s: float, ntypes: int, seed: int = DEFAULT_SEED, zipf_s: float = 1.2,
                  unit: int = 256, kmax: int = 262144):
    """Open-loop trace: Poisson arrival times (us), pack/unpack 50/50, type
    index uniform, requested packed bytes = unit * k with k ~ Zipf(zipf_s)
    rejected above kmax (256 B .. 64 MiB)."""
    g = rng(seed + 17)
    n = int(rate * duration_s * 1.1) + 16
    t = np.cumsum(g.exponential(1e6 / rate, size=n))
    t = t[t < duration_s * 1e6]
    n = t.size
    k = g.zipf(zipf_s, size=n)
    while (k > kmax).any():
        bad = k > kmax
        k[bad] = g.zipf(zipf_s, size=int(bad.sum()))
    return dict(t_us=t, unpack=g.integers(0, 2, size=n).astype(np.int32),
                type_index=g.integers(0, ntypes, size=n).astype(np.int32), target=(unit * k).astype(np.int64))
