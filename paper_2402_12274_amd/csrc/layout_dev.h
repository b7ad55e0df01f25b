// layout_dev.h -- the compiled ("lowered") layout program of a committed
// datatype, as plain data that both host code and gfx950 kernels read, and
// the position arithmetic over it.
//
// A committed type is lowered to
//
//     count loop (stride = extent)
//       x outer loops (regular, over the whole group list)
//         x groups (irregular table: displacement, packed length, shape)
//           x inner loops of the group's shape (regular)
//             x leaf runs of the shape (contiguous byte runs)
//
// which keeps regular layouts O(depth) in size whatever their segment
// count (Derived Datatypes: a face of an Nx x Ny x Nz array is a two-level
// strided vector, not Ny*Nz listed segments) and irregular ones O(blocks).
// A packed-stream byte position is located by one magic-number division
// per regular level and a directory-guided search over the group table;
// the same search by run index bisects segments (MPIX_Type_iov_len).
#pragma once

#include <stdint.h>

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#define MDT_HD __host__ __device__ __forceinline__
#else
#define MDT_HD inline
#endif

namespace mdt {

// Element i of a table in device memory.  In device code the read goes
// through a global-address-space pointer, so it compiles to a global load
// rather than a flat one (flat accesses also count against the LDS wait
// counter, which would make every LDS wait drain outstanding memory reads).
template <class T>
MDT_HD T gld(const T *p, int64_t i)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const __attribute__((address_space(1))) T *)p)[i];
#else
    return p[i];
#endif
}


constexpr int MAXO = 4;   // outer loops
constexpr int MAXI = 4;   // inner loops per shape
constexpr int LEAFI = 8;  // leaf runs stored inline in a shape

// n / d for 0 <= n < 2^63 by one 64x64->128 high multiply and a shift
// (Granlund & Montgomery 1994, "Division by invariant integers using
// multiplication", round-up variant with N = 63).  d == 1 is flagged.
struct MagicDiv {
    uint64_t m;
    uint32_t s;
    uint32_t one;
};

MDT_HD uint64_t mulhi64(uint64_t a, uint64_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

MDT_HD uint64_t magic_div(uint64_t n, const MagicDiv &d)
{
    return d.one ? n : (mulhi64(n, d.m) >> d.s);
}

inline MagicDiv make_magic(uint64_t d)
{
    MagicDiv r{0, 0, 0};
    if (d <= 1) {
        r.one = 1;
        return r;
    }
    // l = ceil(log2 d); m = ceil(2^(63+l) / d) < 2^64; q = mulhi(n, m) >> (l-1)
    uint32_t l = 0;
    while (l < 64 && ((uint64_t)1 << l) < d) l++;
    unsigned __int128 num = (unsigned __int128)1 << (63 + l);
    unsigned __int128 m = (num + d - 1) / d;
    r.m = (uint64_t)m;
    r.s = l - 1;
    return r;
}

// n / d for 0 <= n < 2^31 and 1 <= d < 2^31 with a 32-bit high multiply:
// m = ceil(2^(31+l) / d) < 2^32, q = mulhi(n, m) >> (l-1), l = ceil(log2 d).
struct MagicDiv32 {
    uint32_t m;
    uint32_t s;
    uint32_t one;
};

MDT_HD uint32_t magic_div32(uint32_t n, const MagicDiv32 &d)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return d.one ? n : (__umulhi(n, d.m) >> d.s);
#else
    return d.one ? n : (uint32_t)(((uint64_t)n * d.m) >> 32) >> d.s;
#endif
}

inline MagicDiv32 make_magic32(uint32_t d)
{
    MagicDiv32 r{0, 0, 0};
    if (d <= 1) {
        r.one = 1;
        return r;
    }
    uint32_t l = 0;
    while (l < 32 && ((uint64_t)1 << l) < d) l++;
    uint64_t num = (uint64_t)1 << (31 + l);
    r.m = (uint32_t)((num + d - 1) / d);
    r.s = l - 1;
    return r;
}

struct DevShape {
    int32_t nloops;     // inner loops, outer to inner
    int32_t nleaf;      // leaf runs (0 when varlen)
    int32_t varlen;     // the shape is one run as long as its group
    int32_t implicit0;  // loop 0's count is the group length / span[0]
    int64_t unit;       // packed bytes per innermost iteration (sum of leaf lengths)
    int64_t span[MAXI];    // packed bytes per iteration of loop l
    int64_t stride[MAXI];  // byte stride of loop l
    int64_t cnt[MAXI];     // iteration count of loop l (loop 0: see implicit0)
    int64_t rpi[MAXI];     // runs per iteration of loop l
    MagicDiv dspan[MAXI];
    MagicDiv drpi[MAXI];
    MagicDiv32 dspan32[MAXI];  // valid when small32
    int32_t small32;           // every span < 2^31: positions inside a group fit 32 bits
    int32_t pad_;
    int64_t loff[LEAFI];    // leaf run offsets (inline when nleaf <= LEAFI)
    int64_t llen[LEAFI];
    int64_t lpre[LEAFI + 1];  // leaf prefix: lpre[j] = sum of llen[0..j)
    const int64_t *loff_p;  // leaf arrays when nleaf > LEAFI
    const int64_t *llen_p;
    const int64_t *lpre_p;
};

// Record view: the packed stream is a sequence of equally spaced records
// (element e at byte B0 + e*X), each holding the same leaf runs, U packed
// bytes in total.  Dense record streams (small X/U) are moved by staging a
// tile's typed span in LDS and mapping bytes through per-record tables.
constexpr int32_t REC_MAX_U = 4096;
constexpr int32_t REC_MAX_X = 4096;
constexpr int32_t REC_MIN_RUN = 64;  // the view is used when runs average fewer bytes

struct DevRecords {
    int32_t on;        // 1 when the view applies
    int32_t U;         // packed bytes per record
    int32_t X;         // byte stride of records (> 0)
    int32_t lo, hi;    // a record's bytes lie in [origin + lo, origin + hi)
    int32_t unpack_ok; // hi - lo <= X and no byte of a record is covered twice
    int32_t count1_only; // the view describes element 0 of a count only
    int32_t pad_;
    int64_t B0;        // displacement of record 0's origin
    MagicDiv dU;       // 64-bit divisions by U
    MagicDiv32 dU32;   // 32-bit divisions by U and X
    MagicDiv32 dX32;
    int32_t tile_chunks; // chunks per tile for which the spans fit in LDS
    int32_t lds_bytes;   // dynamic LDS for that tile (spans + table)
    const uint32_t *ptab;  // [U] packed q -> (typed offset - lo) | (run bytes left from q) << 16
    const uint32_t *ttab;  // [X] typed offset d - lo -> q | (run bytes left) << 16 | valid << 31
    // chunk table (pack, U <= REC_CTAB_MAX_U): [U][16] typed offsets, relative
    // to lo of the record holding packed q, of packed bytes q .. q + 15
    const uint32_t *ctab;
    // dword table (unpack, 4 <= X <= REC_DTAB_MAX_X): [X][4] for typed bytes
    // d .. d + 3 (relative to lo; past X they belong to the next record):
    // packed offsets from the record's packed start (+ U in the next record),
    // two 16-bit halves per word, then the mask of bytes the typemap covers
    const uint32_t *dtab;
};

constexpr int32_t REC_CTAB_MAX_U = 256;
constexpr int32_t REC_DTAB_MAX_X = 1024;

enum LayoutKind : int32_t {
    KIND_EMPTY = 0,   // no bytes
    KIND_CONTIG = 1,  // the packed stream is one contiguous run: addr = base + p
    KIND_SINGLE = 2,  // one group, no outer loops
    KIND_MULTI = 3    // group table (optionally under outer loops)
};

struct DevLayout {
    int64_t size;     // packed bytes of one element
    int64_t extent;   // stride between elements of a count
    MagicDiv dsize;
    int32_t kind;
    int32_t nouter;
    int64_t ospan[MAXO];    // packed bytes per iteration of outer loop l
    int64_t ostride[MAXO];
    int64_t ocnt[MAXO];
    int64_t orun[MAXO];     // runs per iteration of outer loop l
    MagicDiv dospan[MAXO];
    MagicDiv dorun[MAXO];
    int64_t G;              // groups
    int64_t gsize;          // packed bytes of the whole group list
    int64_t gruns;          // runs of the whole group list
    int64_t nruns;          // runs of one element
    int64_t gdisp0;         // KIND_SINGLE: displacement of group 0; KIND_CONTIG: address of the run (its leaf offset included)
    int32_t nshapes;
    int32_t dir_shift;      // directory granularity = 1 << dir_shift packed bytes
    int32_t runs_only;      // every group is a single run (varlen shape), no outer loops
    int32_t pad1_;
    int64_t ndir;           // directory entries
    const int64_t *gdisp;   // [G]   group displacement
    const int64_t *gpre;    // [G+1] packed-byte prefix of groups
    const int64_t *grpre;   // [G+1] run prefix of groups
    const int32_t *gshape;  // [G]   shape index (NULL when nshapes == 1)
    const int32_t *gdir;    // [ndir] group containing byte k << dir_shift of the group list
    const DevShape *shapes; // [nshapes]
    DevShape shape0;        // copy of shapes[0]
    DevRecords rec;         // record view (rec.on == 0 when it does not apply)
};

// Result of locating a packed-stream byte position.
struct Loc {
    int64_t addr;  // byte displacement (from the origin) of the located byte
    int64_t rem;   // bytes left in its run, the located byte included
};

// The leaf run holding packed offset q of a shape's innermost body:
// returns its offset, length and packed start.  Inline leaves are scanned
// with static indices only (no pointer into the descriptor is formed, so a
// descriptor passed as a kernel argument stays in the argument segment).
struct Leaf {
    int64_t off, len, pre;
};

MDT_HD Leaf leaf_of(const DevShape &S, uint64_t q)
{
    Leaf r;
    if (S.nleaf > LEAFI) {
        int lo = 0, hi = S.nleaf - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if ((uint64_t)gld(S.lpre_p, mid) <= q) lo = mid; else hi = mid - 1;
        }
        r.off = gld(S.loff_p, lo);
        r.len = gld(S.llen_p, lo);
        r.pre = gld(S.lpre_p, lo);
        return r;
    }
    r.off = S.loff[0];
    r.len = S.llen[0];
    r.pre = 0;
#pragma unroll
    for (int i = 1; i < LEAFI; i++) {
        if (i < S.nleaf && (uint64_t)S.lpre[i] <= q) {
            r.off = S.loff[i];
            r.len = S.llen[i];
            r.pre = S.lpre[i];
        }
    }
    return r;
}

// Leaf run number j (< nleaf): offset and length.
MDT_HD Leaf leaf_at(const DevShape &S, uint64_t j)
{
    Leaf r;
    if (S.nleaf > LEAFI) {
        r.off = gld(S.loff_p, j);
        r.len = gld(S.llen_p, j);
        r.pre = gld(S.lpre_p, j);
        return r;
    }
    r.off = S.loff[0];
    r.len = S.llen[0];
    r.pre = 0;
#pragma unroll
    for (int i = 1; i < LEAFI; i++) {
        if ((uint64_t)i == j) {
            r.off = S.loff[i];
            r.len = S.llen[i];
            r.pre = S.lpre[i];
        }
    }
    return r;
}

// Position q (< 2^31) inside a fixed shape whose spans all fit 32 bits.
MDT_HD Loc locate_in_shape32(const DevShape &S, uint32_t q, int64_t addr)
{
    Loc r;
#pragma unroll
    for (int l = 0; l < MAXI; l++) {
        if (l < S.nloops) {
            uint32_t i = magic_div32(q, S.dspan32[l]);
            q -= i * (uint32_t)S.span[l];
            addr += (int64_t)i * S.stride[l];
        }
    }
    Leaf f = leaf_of(S, q);
    int64_t in = (int64_t)q - f.pre;
    r.addr = addr + f.off + in;
    r.rem = f.len - in;
    return r;
}

// Position q inside one group of shape S (q < group length glen).
MDT_HD Loc locate_in_shape(const DevShape &S, uint64_t q, int64_t glen, int64_t addr)
{
    Loc r;
    if (S.varlen) {
        r.addr = addr + (int64_t)q;
        r.rem = glen - (int64_t)q;
        return r;
    }
#pragma unroll
    for (int l = 0; l < MAXI; l++) {
        if (l < S.nloops) {
            uint64_t i = magic_div(q, S.dspan[l]);
            q -= i * (uint64_t)S.span[l];
            addr += (int64_t)i * S.stride[l];
        }
    }
    Leaf f = leaf_of(S, q);
    int64_t in = (int64_t)q - f.pre;
    r.addr = addr + f.off + in;
    r.rem = f.len - in;
    return r;
}

// Group containing byte q (< gsize) of the group list.
MDT_HD int64_t find_group(const DevLayout &L, uint64_t q)
{
    int64_t k = (int64_t)(q >> L.dir_shift);
    int64_t lo = gld(L.gdir, k);
    int64_t hi = (k + 1 < L.ndir) ? gld(L.gdir, k + 1) : L.G - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if ((uint64_t)gld(L.gpre, mid) <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Locate stream byte p (0 <= p < count*size) of (count x type).  elem1:
// the caller guarantees p < size (only element 0 is touched).
template <int KIND>
MDT_HD Loc locate(const DevLayout &L, uint64_t p, bool elem1 = false)
{
    Loc r;
    if (KIND == KIND_CONTIG) {
        r.addr = L.gdisp0 + (int64_t)p;
        r.rem = INT64_MAX;
        return r;
    }
    uint64_t e = elem1 ? 0 : magic_div(p, L.dsize);
    uint64_t q = p - e * (uint64_t)L.size;
    int64_t addr = (int64_t)e * L.extent;
    if (KIND == KIND_SINGLE) {
        if (L.shape0.small32) return locate_in_shape32(L.shape0, (uint32_t)q, addr + L.gdisp0);
        r = locate_in_shape(L.shape0, q, L.size, addr + L.gdisp0);
        return r;
    }
#pragma unroll
    for (int l = 0; l < MAXO; l++) {
        if (l < L.nouter) {
            uint64_t i = magic_div(q, L.dospan[l]);
            q -= i * (uint64_t)L.ospan[l];
            addr += (int64_t)i * L.ostride[l];
        }
    }
    int64_t g = find_group(L, q);
    int64_t g0 = gld(L.gpre, g);
    int64_t glen = gld(L.gpre, g + 1) - g0;
    // shapes are read from the device table (never from the argument copy)
    const DevShape &S = L.shapes[L.nshapes == 1 ? 0 : gld(L.gshape, g)];
    return locate_in_shape(S, q - (uint64_t)g0, glen, addr + gld(L.gdisp, g));
}

MDT_HD Loc locate_any(const DevLayout &L, uint64_t p)
{
    switch (L.kind) {
    case KIND_CONTIG: return locate<KIND_CONTIG>(L, p);
    case KIND_SINGLE: return locate<KIND_SINGLE>(L, p);
    default: return locate<KIND_MULTI>(L, p);
    }
}

// Run number k (0 <= k < nruns) of one element: its displacement and length.
struct RunInfo {
    int64_t addr;
    int64_t len;
};

MDT_HD RunInfo run_at(const DevLayout &L, uint64_t k)
{
    RunInfo r;
    int64_t addr = 0;
    const DevShape *S;
    int64_t glen;
    if (L.kind == KIND_CONTIG) {
        // one run per element; gdisp0 already includes the run's offset
        r.addr = L.gdisp0;
        r.len = L.size;
        return r;
    }
    if (L.kind == KIND_SINGLE) {
        S = &L.shape0;
        addr = L.gdisp0;
        glen = L.size;
    } else {
#pragma unroll
        for (int l = 0; l < MAXO; l++) {
            if (l < L.nouter) {
                uint64_t i = magic_div(k, L.dorun[l]);
                k -= i * (uint64_t)L.orun[l];
                addr += (int64_t)i * L.ostride[l];
            }
        }
        int64_t lo = 0, hi = L.G - 1;
        while (lo < hi) {
            int64_t mid = (lo + hi + 1) >> 1;
            if ((uint64_t)gld(L.grpre, mid) <= k) lo = mid; else hi = mid - 1;
        }
        k -= (uint64_t)gld(L.grpre, lo);
        addr += gld(L.gdisp, lo);
        glen = gld(L.gpre, lo + 1) - gld(L.gpre, lo);
        S = &L.shapes[L.nshapes == 1 ? 0 : gld(L.gshape, lo)];
    }
    if (S->varlen) {
        r.addr = addr;
        r.len = glen;
        return r;
    }
#pragma unroll
    for (int l = 0; l < MAXI; l++) {
        if (l < S->nloops) {
            uint64_t i = magic_div(k, S->drpi[l]);
            k -= i * (uint64_t)S->rpi[l];
            addr += (int64_t)i * S->stride[l];
        }
    }
    Leaf f = leaf_at(*S, k);
    r.addr = addr + f.off;
    r.len = f.len;
    return r;
}

}  // namespace mdt
