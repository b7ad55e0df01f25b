// xfer.h -- device-side chunk bodies of pack and unpack (gfx950), shared by
// the single-request kernels and the persistent batch kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"
#include "layout_dev.h"

namespace mdt {

// ---------------------------------------------------------------------------
// register-level byte plumbing

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

struct V4 {
    uint32_t w0, w1, w2, w3;
};

// Global-address-space view of a generic pointer into device memory: loads
// and stores through it compile to global_* instructions.  Flat ones would
// also count against the LDS wait counter, so every LDS wait in a tile would
// drain the tile's outstanding memory traffic as well.
#define MDT_G __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ MDT_G T *gptr(T *p)
{
    return (MDT_G T *)p;
}
template <class T>
__device__ __forceinline__ const MDT_G T *gptr(const T *p)
{
    return (const MDT_G T *)p;
}

typedef uint32_t u32x4a1l __attribute__((ext_vector_type(4), aligned(1)));

// 16 bytes at any alignment with one load (global memory takes unaligned
// loads; every byte loaded is one of the 16).  Used where gathers of short
// scattered runs are bound by instructions issued; the chunk kernels keep
// load16, whose alignment cases cost fewer scalar registers there.
__device__ __forceinline__ V4 load16_any(const uint8_t *s)
{
    const u32x4a1l v = *gptr((const u32x4a1l *)s);
    return V4{v.x, v.y, v.z, v.w};
}

// A 16-byte chunk of the packed output: cached or streaming (A.keep).
__device__ __forceinline__ void store_out(const XferArgs &A, uint8_t *dst, const u32x4 &v)
{
    if (A.keep) *gptr((u32x4 *)dst) = v;
    else __builtin_nontemporal_store(v, gptr((u32x4 *)dst));
}

// Byte / dword extraction at a variable byte position of the chunk, as
// 128-bit shifts (funnel shifts in registers; an indexed select would be
// turned into a per-lane memory array).
__device__ __forceinline__ unsigned __int128 as128(const V4 &a)
{
    return ((unsigned __int128)a.w3 << 96) | ((unsigned __int128)a.w2 << 64) | ((unsigned __int128)a.w1 << 32) |
           (unsigned __int128)a.w0;
}

__device__ __forceinline__ uint32_t byte_at(const V4 &a, int pos)
{
    return (uint32_t)(as128(a) >> (8 * pos)) & 0xffu;
}

// 4 bytes starting at byte pos (0 <= pos <= 12) of the 16-byte chunk
__device__ __forceinline__ uint32_t dword_at(const V4 &a, int pos) { return (uint32_t)(as128(a) >> (8 * pos)); }

// 16 bytes from an arbitrarily aligned source; every dword loaded holds at
// least one of the 16 bytes, so no access leaves the source's pages.  An
// aligned load streams past the caches unless CACHED.
template <bool CACHED = false>
__device__ __forceinline__ V4 load16(const uint8_t *s)
{
    uintptr_t u = (uintptr_t)s;
    V4 r;
    if ((u & 15) == 0) {
        u32x4 v = CACHED ? *gptr((const u32x4 *)s) : __builtin_nontemporal_load(gptr((const u32x4 *)s));
        r.w0 = v.x; r.w1 = v.y; r.w2 = v.z; r.w3 = v.w;
    } else if ((u & 7) == 0) {
        const MDT_G u32x2 *p = gptr((const u32x2 *)s);
        u32x2 a = p[0], b = p[1];
        r.w0 = a.x; r.w1 = a.y; r.w2 = b.x; r.w3 = b.y;
    } else if ((u & 3) == 0) {
        const MDT_G uint32_t *p = gptr((const uint32_t *)s);
        r.w0 = p[0]; r.w1 = p[1]; r.w2 = p[2]; r.w3 = p[3];
    } else {
        const MDT_G uint32_t *p = gptr((const uint32_t *)(u & ~(uintptr_t)3));
        uint32_t sh = (uint32_t)(u & 3);
        uint32_t d0 = p[0], d1 = p[1], d2 = p[2], d3 = p[3], d4 = p[4];
        r.w0 = __builtin_amdgcn_alignbyte(d1, d0, sh);
        r.w1 = __builtin_amdgcn_alignbyte(d2, d1, sh);
        r.w2 = __builtin_amdgcn_alignbyte(d3, d2, sh);
        r.w3 = __builtin_amdgcn_alignbyte(d4, d3, sh);
    }
    return r;
}

// The part of chunk word t (bytes 4t..4t+3) that bytes s[0..n), placed at
// chunk positions [k, k+n), contribute.
__device__ __forceinline__ uint32_t gather_word(int t, int k, const uint8_t *s, int n)
{
    int a = max(4 * t, k), b = min(4 * t + 4, k + n);
    if (a >= b) return 0u;
    uintptr_t u = (uintptr_t)(s + (a - k));
    const MDT_G uint32_t *p = gptr((const uint32_t *)(u & ~(uintptr_t)3));
    uint32_t sh = (uint32_t)(u & 3);
    int cnt = b - a;
    uint32_t lo = p[0];
    uint32_t hi = ((int)sh + cnt > 4) ? p[1] : 0u;
    uint32_t v = __builtin_amdgcn_alignbyte(hi, lo, sh);
    uint32_t m = cnt >= 4 ? 0xffffffffu : ((1u << (8 * cnt)) - 1u);
    return (v & m) << (8 * (a - 4 * t));
}

// OR bytes s[0..n) into chunk positions [k, k+n)  (n < 16 or k > 0)
__device__ __forceinline__ void gather_part(V4 &acc, int k, const uint8_t *s, int n)
{
    acc.w0 |= gather_word(0, k, s, n);
    acc.w1 |= gather_word(1, k, s, n);
    acc.w2 |= gather_word(2, k, s, n);
    acc.w3 |= gather_word(3, k, s, n);
}

typedef uint32_t u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));

// OR bytes s[0..n) (0 < n <= 16 - k) into chunk positions [k, k+n) with one
// 16-byte load from the dword holding s[0], and one more dword when the
// bytes run past it: one or two memory instructions per piece instead of
// one or two per word (a gather of scattered runs is bound by instructions
// issued, each touching a different line per lane).  The bytes loaded
// beyond s[0..n) lie in the same 4 KiB page as s[0], so no access leaves a
// mapped page; within 20 bytes of a page end the word-by-word gather is
// used instead.
__device__ __forceinline__ void gather_piece(V4 &acc, int k, const uint8_t *s, int n)
{
    const uintptr_t u = (uintptr_t)s;
    const uintptr_t a4 = u & ~(uintptr_t)3;
    if ((a4 & 4095) > 4096 - 20) {
        gather_part(acc, k, s, n);
        return;
    }
    const int sh = (int)(u & 3);
    const u32x4a4 w = *gptr((const u32x4a4 *)a4);
    const uint32_t e = sh + n > 16 ? *gptr((const uint32_t *)(a4 + 16)) : 0u;
    unsigned __int128 v = (((unsigned __int128)w.w << 96) | ((unsigned __int128)w.z << 64) |
                           ((unsigned __int128)w.y << 32) | (unsigned __int128)w.x) >>
                          (8 * sh);
    if (sh) v |= (unsigned __int128)e << (8 * (16 - sh));
    if (n < 16) v &= ((unsigned __int128)1 << (8 * n)) - 1;
    v <<= 8 * k;
    acc.w0 |= (uint32_t)v;
    acc.w1 |= (uint32_t)(v >> 32);
    acc.w2 |= (uint32_t)(v >> 64);
    acc.w3 |= (uint32_t)(v >> 96);
}

typedef uint32_t u32x4a1 __attribute__((ext_vector_type(4), aligned(1)));
typedef uint32_t u32x2a1 __attribute__((ext_vector_type(2), aligned(1)));
typedef uint32_t u32a1 __attribute__((aligned(1)));
typedef uint16_t u16a1 __attribute__((aligned(1)));

// write chunk bytes [k, k+n) to d[0..n): only those bytes are stored.  The
// piece goes out as at most one store per set bit of n (16, 8, 4, 2 and 1
// bytes), at any alignment (global memory takes unaligned accesses; each
// store covers piece bytes only, so neighbouring bytes are never written):
// a scatter of scattered short runs is bound by the stores issued.
__device__ __forceinline__ void scatter(const V4 &acc, int k, uint8_t *d, int n)
{
    if (n == 16) {
        if (((uintptr_t)d & 15) == 0) *gptr((u32x4 *)d) = u32x4{acc.w0, acc.w1, acc.w2, acc.w3};
        else *gptr((u32x4a1 *)d) = u32x4a1{acc.w0, acc.w1, acc.w2, acc.w3};
        return;
    }
    unsigned __int128 v = as128(acc) >> (8 * k);
    int o = 0;
    if (n & 8) {
        *gptr((u32x2a1 *)(d + o)) = u32x2a1{(uint32_t)v, (uint32_t)(v >> 32)};
        v >>= 64;
        o += 8;
    }
    if (n & 4) {
        *gptr((u32a1 *)(d + o)) = (uint32_t)v;
        v >>= 32;
        o += 4;
    }
    if (n & 2) {
        *gptr((u16a1 *)(d + o)) = (uint16_t)v;
        v >>= 16;
        o += 2;
    }
    if (n & 1) *gptr(d + o) = (uint8_t)v;
}

// ---------------------------------------------------------------------------
// chunk bodies

template <int KIND, bool CACHED>
__device__ __forceinline__ void pack_chunk(const DevLayout &L, const XferArgs &A, int64_t c)
{
    int64_t lo = 16 * c - A.head;
    int64_t a = lo > 0 ? lo : 0;
    int64_t b = lo + 16 < A.nbytes ? lo + 16 : A.nbytes;
    int k = (int)(a - lo);
    int n = (int)(b - a);
    uint64_t p = (uint64_t)(A.off + a);
    V4 acc = {0u, 0u, 0u, 0u};
    const uint8_t *src = A.typed;
    Loc l = locate<KIND>(L, p, A.elem1);
    if (n == 16 && l.rem >= 16) {
        acc = load16<CACHED>(src + l.addr);
    } else {
        // the first two runs are located before either is read, so their
        // loads are in flight together (chunks of small blocks mostly hold
        // two runs); further runs follow one at a time
        int take = l.rem < n ? (int)l.rem : n;
        int take2 = 0;
        Loc l2 = l;
        if (take > 0 && take < n) {
            l2 = locate<KIND>(L, p + (uint64_t)take, A.elem1);
            take2 = l2.rem < n - take ? (int)l2.rem : n - take;
            if (take2 < 0) take2 = 0;
        }
        if (take > 0) gather_piece(acc, k, src + l.addr, take);
        if (take2 > 0) gather_piece(acc, k + take, src + l2.addr, take2);
        if (take > 0 && take2 > 0 && take + take2 < n) {
            p += (uint64_t)(take + take2);
            k += take + take2;
            n -= take + take2;
            l = locate<KIND>(L, p, A.elem1);
            for (;;) {
                int t = l.rem < n ? (int)l.rem : n;
                if (t <= 0) break;  // unreachable for a well-formed layout; never spin
                gather_piece(acc, k, src + l.addr, t);
                p += t;
                k += t;
                n -= t;
                if (n <= 0) break;
                l = locate<KIND>(L, p, A.elem1);
            }
        }
    }
    uint8_t *dst = A.packed - A.head + 16 * c;
    if (a == lo && b == lo + 16) {
        u32x4 v = {acc.w0, acc.w1, acc.w2, acc.w3};
        store_out(A, dst, v);
    } else {
        for (int i = (int)(a - lo); i < (int)(b - lo); i++) gptr(dst)[i] = (uint8_t)byte_at(acc, i);
    }
}

template <int KIND>
__device__ __forceinline__ void unpack_chunk(const DevLayout &L, const XferArgs &A, int64_t c)
{
    int64_t lo = 16 * c - A.head;
    int64_t a = lo > 0 ? lo : 0;
    int64_t b = lo + 16 < A.nbytes ? lo + 16 : A.nbytes;
    int k = (int)(a - lo);
    int n = (int)(b - a);
    // the aligned 16-byte block holding this chunk's packed bytes
    const uint8_t *in = A.packed - A.head + 16 * c;
    u32x4 v = __builtin_nontemporal_load(gptr((const u32x4 *)in));
    V4 acc = {v.x, v.y, v.z, v.w};
    uint64_t p = (uint64_t)(A.off + a);
    uint8_t *dst = const_cast<uint8_t *>(A.typed);
    Loc l = locate<KIND>(L, p, A.elem1);
    for (;;) {
        int take = l.rem < n ? (int)l.rem : n;
        if (take <= 0) break;  // unreachable for a well-formed layout; never spin
        scatter(acc, k, dst + l.addr, take);
        p += take;
        k += take;
        n -= take;
        if (n <= 0) break;
        l = locate<KIND>(L, p, A.elem1);
    }
}

// Load chunk c whole when its bytes lie in one run or in two dword-aligned
// runs; false when it needs the general body (or lies outside the tile).
template <int KIND, bool CACHED>
__device__ __forceinline__ bool pack_first(const DevLayout &L, const XferArgs &A, int64_t c, int64_t cend, V4 &acc)
{
    int64_t lo = 16 * c - A.head;
    if (c < cend && lo >= 0 && lo + 16 <= A.nbytes) {
        Loc l = locate<KIND>(L, (uint64_t)(A.off + lo), A.elem1);
        if (l.rem >= 16) {
            acc = load16<CACHED>(A.typed + l.addr);
            return true;
        }
        // two runs split on a dword boundary, both dword aligned (blocks of
        // float64 or int32 at a stride): four independent dword loads, each
        // from whichever run holds that word
        const uintptr_t a1 = (uintptr_t)(A.typed + l.addr);
        const int t1 = (int)l.rem;
        if (((a1 | (uintptr_t)t1) & 3) == 0) {
            Loc l2 = locate<KIND>(L, (uint64_t)(A.off + lo + t1), A.elem1);
            const uintptr_t a2 = (uintptr_t)(A.typed + l2.addr) - (uintptr_t)t1;  // chunk byte j of run 2 at a2 + j
            if (l2.rem >= 16 - t1 && (a2 & 3) == 0) {
                if (t1 == 8 && ((a1 | a2) & 7) == 0) {
                    // two 8-byte blocks (float64 at a stride): one request each
                    const u32x2 x = *gptr((const u32x2 *)a1);
                    const u32x2 y = *gptr((const u32x2 *)(a2 + 8));
                    acc = V4{x.x, x.y, y.x, y.y};
                    return true;
                }
                acc.w0 = *gptr((const uint32_t *)(0 < t1 ? a1 : a2));
                acc.w1 = *gptr((const uint32_t *)(4 < t1 ? a1 + 4 : a2 + 4));
                acc.w2 = *gptr((const uint32_t *)(8 < t1 ? a1 + 8 : a2 + 8));
                acc.w3 = *gptr((const uint32_t *)(12 < t1 ? a1 + 12 : a2 + 12));
                return true;
            }
        }
    }
    return false;
}

__device__ __forceinline__ void store_chunk(const XferArgs &A, int64_t c, const V4 &acc)
{
    u32x4 v = {acc.w0, acc.w1, acc.w2, acc.w3};
    store_out(A, (A.packed - A.head + 16 * c), v);
}

// Whole tile inside one run: the typed address of packed byte lo (relative
// to the packed start) is base + lo.  Returns false when the tile's bytes
// span several runs (or the layout is contiguous, which needs no test).
template <int KIND>
__device__ __forceinline__ bool tile_in_one_run(const DevLayout &L, const XferArgs &A, int64_t c0, int64_t cend,
                                                int64_t &base)
{
    const int64_t P_lo = max(16 * c0 - A.head, (int64_t)0);
    const int64_t P_hi = min(16 * cend - A.head, A.nbytes);
    Loc l = locate<KIND>(L, (uint64_t)(A.off + P_lo), A.elem1);
    base = l.addr - P_lo;
    return l.rem >= P_hi - P_lo;
}

template <int KIND>
__device__ __forceinline__ void pack_tile_run(const XferArgs &A, int64_t c0, int64_t cend, int64_t base)
{
    const int64_t c = c0 + threadIdx.x;
    V4 a0 = {0u, 0u, 0u, 0u}, a1 = a0, a2 = a0, a3 = a0;
    uint32_t full = 0;
#define MDT_RUN_LOAD(k, a)                                                   \
    {                                                                        \
        int64_t ck = c + 256 * (k), lo = 16 * ck - A.head;                   \
        if (ck < cend && lo >= 0 && lo + 16 <= A.nbytes) {                   \
            a = load16(A.typed + base + lo);                                 \
            full |= 1u << (k);                                               \
        }                                                                    \
    }
    MDT_RUN_LOAD(0, a0) MDT_RUN_LOAD(1, a1) MDT_RUN_LOAD(2, a2) MDT_RUN_LOAD(3, a3)
#undef MDT_RUN_LOAD
    if (full & 1u) store_chunk(A, c, a0);
    if (full & 2u) store_chunk(A, c + 256, a1);
    if (full & 4u) store_chunk(A, c + 512, a2);
    if (full & 8u) store_chunk(A, c + 768, a3);
#pragma unroll 1
    for (int k = 0; k < 4; k++) {
        int64_t ck = c + 256 * k;
        if (ck >= cend || ((full >> k) & 1u)) continue;
        // edge chunk of the transfer: byte by byte
        const int64_t lo = 16 * ck - A.head;
        const int64_t a = lo > 0 ? lo : 0, b = lo + 16 < A.nbytes ? lo + 16 : A.nbytes;
        uint8_t *dst = A.packed - A.head + 16 * ck;
        for (int64_t j = a; j < b; j++) gptr(dst)[j - lo] = gptr(A.typed)[base + j];
    }
}

template <int KIND>
__device__ __forceinline__ void unpack_tile_run(const XferArgs &A, int64_t c0, int64_t cend, int64_t base)
{
    const int64_t c = c0 + threadIdx.x;
    uint8_t *typed = const_cast<uint8_t *>(A.typed);
    V4 a0 = {0u, 0u, 0u, 0u}, a1 = a0, a2 = a0, a3 = a0;
    uint32_t full = 0;
#define MDT_RUN_LOAD(k, a)                                                               \
    {                                                                                    \
        int64_t ck = c + 256 * (k), lo = 16 * ck - A.head;                               \
        if (ck < cend && lo >= 0 && lo + 16 <= A.nbytes) {                               \
            u32x4 v = __builtin_nontemporal_load(gptr((const u32x4 *)(A.packed - A.head + 16 * ck))); \
            a = V4{v.x, v.y, v.z, v.w};                                                  \
            full |= 1u << (k);                                                           \
        }                                                                                \
    }
    MDT_RUN_LOAD(0, a0) MDT_RUN_LOAD(1, a1) MDT_RUN_LOAD(2, a2) MDT_RUN_LOAD(3, a3)
#undef MDT_RUN_LOAD
    if (full & 1u) scatter(a0, 0, typed + base + (16 * c - A.head), 16);
    if (full & 2u) scatter(a1, 0, typed + base + (16 * (c + 256) - A.head), 16);
    if (full & 4u) scatter(a2, 0, typed + base + (16 * (c + 512) - A.head), 16);
    if (full & 8u) scatter(a3, 0, typed + base + (16 * (c + 768) - A.head), 16);
#pragma unroll 1
    for (int k = 0; k < 4; k++) {
        int64_t ck = c + 256 * k;
        if (ck >= cend || ((full >> k) & 1u)) continue;
        const int64_t lo = 16 * ck - A.head;
        const int64_t a = lo > 0 ? lo : 0, b = lo + 16 < A.nbytes ? lo + 16 : A.nbytes;
        const uint8_t *src = A.packed - A.head + 16 * ck;
        for (int64_t j = a; j < b; j++) gptr(typed)[base + j] = gptr(src)[j - lo];
    }
}

// A lane's chunks c0 + lane + 256k (k < 4) of a tile, loads first: every
// chunk whose 16 bytes lie in one run, or in two dword-aligned runs, is
// loaded before any store is issued, so up to four gathers per lane are in
// flight at once.  The other chunks then take the general body, one at a
// time.  A tile that lies inside one run is a plain copy.  CACHED: the
// gathers load through the caches (a launch over runs shorter than a line,
// whose lines other runs read soon after), else they stream.
template <int KIND, bool CACHED = false>
__device__ __forceinline__ void pack_tile4(const DevLayout &L, const XferArgs &A, int64_t c0, int64_t cend)
{
    if (KIND != KIND_CONTIG) {
        int64_t base;
        if (tile_in_one_run<KIND>(L, A, c0, cend, base)) {
            pack_tile_run<KIND>(A, c0, cend, base);
            return;
        }
    }
    const int64_t c = c0 + threadIdx.x;
    V4 a0 = {0u, 0u, 0u, 0u}, a1 = a0, a2 = a0, a3 = a0;
    uint32_t fast = (uint32_t)pack_first<KIND, CACHED>(L, A, c, cend, a0) |
                    (uint32_t)pack_first<KIND, CACHED>(L, A, c + 256, cend, a1) << 1 |
                    (uint32_t)pack_first<KIND, CACHED>(L, A, c + 512, cend, a2) << 2 |
                    (uint32_t)pack_first<KIND, CACHED>(L, A, c + 768, cend, a3) << 3;
    if (fast & 1u) store_chunk(A, c, a0);
    if (fast & 2u) store_chunk(A, c + 256, a1);
    if (fast & 4u) store_chunk(A, c + 512, a2);
    if (fast & 8u) store_chunk(A, c + 768, a3);
#pragma unroll 1
    for (int k = 0; k < 4; k++) {
        int64_t ck = c + 256 * k;
        if (ck < cend && !((fast >> k) & 1u)) pack_chunk<KIND, CACHED>(L, A, ck);
    }
}

// Load chunk c's packed 16 bytes and locate its first byte; false for a
// chunk outside the tile or one that the transfer's range clips.
template <int KIND>
__device__ __forceinline__ bool unpack_first(const DevLayout &L, const XferArgs &A, int64_t c, int64_t cend, V4 &acc,
                                             Loc &loc)
{
    int64_t lo = 16 * c - A.head;
    if (c < cend && lo >= 0 && lo + 16 <= A.nbytes) {
        u32x4 v = __builtin_nontemporal_load(gptr((const u32x4 *)(A.packed - A.head + 16 * c)));
        acc = V4{v.x, v.y, v.z, v.w};
        loc = locate<KIND>(L, (uint64_t)(A.off + lo), A.elem1);
        return true;
    }
    return false;
}

// Store a whole chunk (stream bytes [p, p + 16), first run l) to the typed
// side, run by run.  Stores do not wait, so a lane's chunks overlap.
template <int KIND>
__device__ __forceinline__ void scatter_chunk(const DevLayout &L, const XferArgs &A, uint64_t p, Loc l, const V4 &acc)
{
    uint8_t *dst = const_cast<uint8_t *>(A.typed);
    if (l.rem >= 16) {
        scatter(acc, 0, dst + l.addr, 16);
        return;
    }
    int k = 0;
    for (;;) {
        int take = l.rem < 16 - k ? (int)l.rem : 16 - k;
        if (take <= 0) break;  // unreachable for a well-formed layout; never spin
        scatter(acc, k, dst + l.addr, take);
        k += take;
        if (k >= 16) break;
        l = locate<KIND>(L, p + (uint64_t)k, A.elem1);
    }
}

// A lane's chunks c0 + lane + 256k (k < 4) of a tile: all four packed loads
// are issued first, then each whole chunk is scattered from its loaded value
// (stores only, so nothing waits between chunks).  Chunks clipped by the
// transfer's range take the general body.  A tile that lies inside one run
// is a plain copy.
template <int KIND>
__device__ __forceinline__ void unpack_tile4(const DevLayout &L, const XferArgs &A, int64_t c0, int64_t cend)
{
    if (KIND != KIND_CONTIG) {
        int64_t base;
        if (tile_in_one_run<KIND>(L, A, c0, cend, base)) {
            unpack_tile_run<KIND>(A, c0, cend, base);
            return;
        }
    }
    const int64_t c = c0 + threadIdx.x;
    V4 a0 = {0u, 0u, 0u, 0u}, a1 = a0, a2 = a0, a3 = a0;
    Loc l0 = {0, 0}, l1 = l0, l2 = l0, l3 = l0;
    uint32_t whole = (uint32_t)unpack_first<KIND>(L, A, c, cend, a0, l0) |
                     (uint32_t)unpack_first<KIND>(L, A, c + 256, cend, a1, l1) << 1 |
                     (uint32_t)unpack_first<KIND>(L, A, c + 512, cend, a2, l2) << 2 |
                     (uint32_t)unpack_first<KIND>(L, A, c + 768, cend, a3, l3) << 3;
    const uint64_t p = (uint64_t)(A.off + 16 * c - A.head);
    if (whole & 1u) scatter_chunk<KIND>(L, A, p, l0, a0);
    if (whole & 2u) scatter_chunk<KIND>(L, A, p + 4096, l1, a1);
    if (whole & 4u) scatter_chunk<KIND>(L, A, p + 8192, l2, a2);
    if (whole & 8u) scatter_chunk<KIND>(L, A, p + 12288, l3, a3);
#pragma unroll 1
    for (int k = 0; k < 4; k++) {
        int64_t ck = c + 256 * k;
        if (ck < cend && !((whole >> k) & 1u)) unpack_chunk<KIND>(L, A, ck);
    }
}



// ---------------------------------------------------------------------------
// typed copy: a chunk of the stream gathered from one layout and scattered
// to another, with no packed buffer in between

// Stream bytes [p, p + n) (n <= 16) of layout L at origin base, as chunk
// bytes [0, n).
template <int KIND>
__device__ __forceinline__ V4 gather_stream(const DevLayout &L, const uint8_t *base, uint64_t p, int n, bool elem1)
{
    Loc l = locate<KIND>(L, p, elem1);
    if (n == 16 && l.rem >= 16) return load16(base + l.addr);
    V4 acc = {0u, 0u, 0u, 0u};
    int k = 0;
    for (;;) {
        int take = l.rem < n ? (int)l.rem : n;
        if (take <= 0) break;  // unreachable for a well-formed layout; never spin
        gather_part(acc, k, base + l.addr, take);
        p += take;
        k += take;
        n -= take;
        if (n <= 0) break;
        l = locate<KIND>(L, p, elem1);
    }
    return acc;
}

// Chunk bytes [0, n) to stream bytes [p, p + n) of layout L at origin base.
template <int KIND>
__device__ __forceinline__ void scatter_stream(const DevLayout &L, uint8_t *base, uint64_t p, int n, const V4 &acc,
                                               bool elem1)
{
    Loc l = locate<KIND>(L, p, elem1);
    int k = 0;
    for (;;) {
        int take = l.rem < n ? (int)l.rem : n;
        if (take <= 0) break;  // unreachable for a well-formed layout; never spin
        scatter(acc, k, base + l.addr, take);
        p += take;
        k += take;
        n -= take;
        if (n <= 0) break;
        l = locate<KIND>(L, p, elem1);
    }
}

// A lane's chunks c0 + lane + 256u (u < 4) of a copy tile: all four are
// gathered before any is scattered, so their loads are in flight together.
template <int KS, int KD>
__device__ __forceinline__ void copy_tile4(const DevLayout &Ls, const DevLayout &Ld, const CopyArgs &A, int64_t c0,
                                           int64_t cend)
{
    V4 acc0 = {0u, 0u, 0u, 0u}, acc1 = acc0, acc2 = acc0, acc3 = acc0;
    const int64_t c = c0 + threadIdx.x;
#define MDT_COPY_N(u) (int)min((int64_t)16, A.nbytes - 16 * (c + 256 * (u)))
#define MDT_COPY_P(u) (uint64_t)(A.off + 16 * (c + 256 * (u)))
    if (c < cend) acc0 = gather_stream<KS>(Ls, A.src, MDT_COPY_P(0), MDT_COPY_N(0), A.src_elem1);
    if (c + 256 < cend) acc1 = gather_stream<KS>(Ls, A.src, MDT_COPY_P(1), MDT_COPY_N(1), A.src_elem1);
    if (c + 512 < cend) acc2 = gather_stream<KS>(Ls, A.src, MDT_COPY_P(2), MDT_COPY_N(2), A.src_elem1);
    if (c + 768 < cend) acc3 = gather_stream<KS>(Ls, A.src, MDT_COPY_P(3), MDT_COPY_N(3), A.src_elem1);
    if (c < cend) scatter_stream<KD>(Ld, A.dst, MDT_COPY_P(0), MDT_COPY_N(0), acc0, A.dst_elem1);
    if (c + 256 < cend) scatter_stream<KD>(Ld, A.dst, MDT_COPY_P(1), MDT_COPY_N(1), acc1, A.dst_elem1);
    if (c + 512 < cend) scatter_stream<KD>(Ld, A.dst, MDT_COPY_P(2), MDT_COPY_N(2), acc2, A.dst_elem1);
    if (c + 768 < cend) scatter_stream<KD>(Ld, A.dst, MDT_COPY_P(3), MDT_COPY_N(3), acc3, A.dst_elem1);
#undef MDT_COPY_N
#undef MDT_COPY_P
}

}  // namespace mdt

namespace mdt {

// ---------------------------------------------------------------------------
// dense record streams: stage the tile's typed span (pack) or packed bytes
// (unpack) in LDS with coalesced 16-byte loads, then move every byte through
// the per-record tables with 32-bit arithmetic.  The packed side is stored
// as whole 16-byte chunks (pack) and the typed side as naturally aligned
// dwords covering only typemap bytes (unpack: gaps are never written).

// 4 bytes from byte offset `off` of an LDS buffer (two aligned reads; the
// buffer has a dword of slack at its end)
__device__ __forceinline__ uint32_t lds_u32(const uint8_t *lds, uint32_t off)
{
    const uint32_t *p = (const uint32_t *)(lds + (off & ~3u));
    return __builtin_amdgcn_alignbyte(p[1], p[0], off & 3u);
}

__device__ __forceinline__ uint32_t lds_u8(const uint8_t *lds, uint32_t off) { return lds[off]; }

// Copy [g_lo, g_hi) rounded out to 16-byte blocks into LDS; returns the LDS
// offset of g_lo.  Every block read holds at least one byte of the range.
__device__ __forceinline__ uint32_t stage_span(uint8_t *lds, const uint8_t *g_lo, const uint8_t *g_hi)
{
    uintptr_t a = (uintptr_t)g_lo & ~(uintptr_t)15;
    uintptr_t b = ((uintptr_t)g_hi + 15) & ~(uintptr_t)15;
    uint32_t nv = (uint32_t)((b - a) >> 4);
    for (uint32_t i = threadIdx.x; i < nv; i += blockDim.x) {
        u32x4 v = __builtin_nontemporal_load(gptr((const u32x4 *)(a + 16 * (uintptr_t)i)));
        *(u32x4 *)(lds + 16 * i) = v;
    }
    return (uint32_t)((uintptr_t)g_lo - a);
}

// Next packed word of a dense record stream: q is the packed offset inside
// record er (relative to the tile's first record); both advance by 4.
__device__ __forceinline__ uint32_t dense_word(const uint32_t *tab, const uint8_t *span, uint32_t base, uint32_t X,
                                               uint32_t U, uint32_t &q, uint32_t &er)
{
    uint32_t e = tab[q];
    if ((e >> 16) >= 4u) {
        uint32_t w = lds_u32(span, base + er * X + (e & 0xffffu));
        q += 4;
        if (q == U) {
            q = 0;
            er++;
        }
        return w;
    }
    uint32_t v = 0;
    for (int i = 0; i < 4; i++) {
        uint32_t ei = tab[q];
        v |= lds_u8(span, base + er * X + (ei & 0xffffu)) << (8 * i);
        if (++q == U) {
            q = 0;
            er++;
        }
    }
    return v;
}

// Pack chunks [c0, c1) of A (a tile) with the record view of L and its byte
// table.  `lds` holds rec.lds_bytes of dynamic shared memory.
__device__ __forceinline__ void dense_pack_tile_b(const DevLayout &L, const XferArgs &A, int64_t c0, int64_t c1,
                                                uint8_t *lds)
{
    const DevRecords &R = L.rec;
    const int64_t P_lo = max(16 * c0 - A.head, (int64_t)0);
    const int64_t P_hi = min(16 * c1 - A.head, A.nbytes);
    const uint64_t s_lo = (uint64_t)(A.off + P_lo);
    const uint64_t e0 = magic_div(s_lo, R.dU);
    const uint64_t e1 = magic_div((uint64_t)(A.off + P_hi - 1), R.dU);
    const int64_t t_lo = R.B0 + (int64_t)e0 * R.X + R.lo;
    const int64_t t_hi = R.B0 + (int64_t)e1 * R.X + R.hi;
    uint32_t *tab = (uint32_t *)lds;
    uint8_t *span = lds + ((4 * (uint32_t)R.U + 15) & ~15u);
    for (int q = threadIdx.x; q < R.U; q += blockDim.x) tab[q] = gld(R.ptab, q);
    const uint32_t base = stage_span(span, A.typed + t_lo, A.typed + t_hi);
    __syncthreads();
    const uint32_t q0 = (uint32_t)(s_lo - e0 * (uint64_t)R.U);  // position of s_lo in record e0
    const uint32_t U = (uint32_t)R.U, X = (uint32_t)R.X;
    for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
        const int64_t lo = 16 * c - A.head;
        const int64_t a = lo > 0 ? lo : 0;
        const int64_t b = lo + 16 < A.nbytes ? lo + 16 : A.nbytes;
        // record and offset of chunk byte a, relative to record e0
        uint32_t rel = (uint32_t)(a - P_lo) + q0;
        uint32_t er = magic_div32(rel, R.dU32);
        uint32_t q = rel - er * U;
        if (a == lo && b == lo + 16) {
            uint32_t w0 = dense_word(tab, span, base, X, U, q, er);
            uint32_t w1 = dense_word(tab, span, base, X, U, q, er);
            uint32_t w2 = dense_word(tab, span, base, X, U, q, er);
            uint32_t w3 = dense_word(tab, span, base, X, U, q, er);
            u32x4 v = {w0, w1, w2, w3};
            store_out(A, (A.packed - A.head + 16 * c), v);
        } else {
            uint8_t *dst = A.packed - A.head + 16 * c;
            for (int i = (int)(a - lo); i < (int)(b - lo); i++) {
                uint32_t ei = tab[q];
                gptr(dst)[i] = (uint8_t)lds_u8(span, base + er * X + (ei & 0xffffu));
                if (++q == U) { q = 0; er++; }
            }
        }
    }
}

// Unpack chunks [c0, c1) of A (a tile) with the byte table: the packed tile
// goes to LDS, then the lanes walk the typed span dword by dword and store
// the typemap bytes that belong to this tile.
__device__ __forceinline__ void dense_unpack_tile_b(const DevLayout &L, const XferArgs &A, int64_t c0, int64_t c1,
                                                  uint8_t *lds)
{
    const DevRecords &R = L.rec;
    const int64_t P_lo = max(16 * c0 - A.head, (int64_t)0);
    const int64_t P_hi = min(16 * c1 - A.head, A.nbytes);
    const uint64_t s_lo = (uint64_t)(A.off + P_lo);
    const uint64_t e0 = magic_div(s_lo, R.dU);
    const uint64_t e1 = magic_div((uint64_t)(A.off + P_hi - 1), R.dU);
    const int64_t t_lo = R.B0 + (int64_t)e0 * R.X + R.lo;
    const int64_t t_hi = R.B0 + (int64_t)e1 * R.X + R.hi;
    uint32_t *tab = (uint32_t *)lds;
    uint8_t *pk = lds + ((4 * (uint32_t)R.X + 15) & ~15u);
    for (int d = threadIdx.x; d < R.X; d += blockDim.x) tab[d] = gld(R.ttab, d);
    const uint32_t pbase = stage_span(pk, A.packed + P_lo, A.packed + P_hi);
    __syncthreads();
    const uint32_t U = (uint32_t)R.U, X = (uint32_t)R.X;
    const uint32_t q0 = (uint32_t)(s_lo - e0 * (uint64_t)U);  // packed position of s_lo in record e0
    const uint32_t npk = (uint32_t)(P_hi - P_lo);             // packed bytes of this tile
    uint8_t *t0 = const_cast<uint8_t *>(A.typed) + t_lo;      // typed byte of (record e0, offset lo)
    const uintptr_t d_lo = (uintptr_t)t0 & ~(uintptr_t)3;
    const uint32_t skew = (uint32_t)((uintptr_t)t0 - d_lo);   // bytes of the first dword before t0
    const uint32_t tspan = (uint32_t)(t_hi - t_lo);
    const uint32_t ndw = (skew + tspan + 3) >> 2;
    for (uint32_t j = threadIdx.x; j < ndw; j += blockDim.x) {
        uint32_t *D = (uint32_t *)(d_lo + 4 * (uintptr_t)j);
        int32_t r0 = (int32_t)(4 * j) - (int32_t)skew;  // typed offset of the dword from t0
        if (r0 >= 0 && (uint32_t)r0 + 4 <= tspan) {
            uint32_t er = magic_div32((uint32_t)r0, R.dX32);
            uint32_t d = (uint32_t)r0 - er * X;
            uint32_t e = tab[d];
            // packed offset in this tile = er*U + q - q0
            int32_t p = (int32_t)(er * U + (e & 0xffffu)) - (int32_t)q0;
            if ((e & 0x80000000u) && ((e >> 16) & 0x7fffu) >= 4u && p >= 0 && (uint32_t)p + 4 <= npk) {
                *gptr(D) = lds_u32(pk, pbase + (uint32_t)p);
                continue;
            }
        }
        // partial dword: byte by byte
        uint8_t *Db = (uint8_t *)D;
        for (int i = 0; i < 4; i++) {
            int32_t r = r0 + i;
            if (r < 0 || (uint32_t)r >= tspan) continue;
            uint32_t er = magic_div32((uint32_t)r, R.dX32);
            uint32_t d = (uint32_t)r - er * X;
            uint32_t e = tab[d];
            if (!(e & 0x80000000u)) continue;
            int32_t p = (int32_t)(er * U + (e & 0xffffu)) - (int32_t)q0;
            if (p < 0 || (uint32_t)p >= npk) continue;
            gptr(Db)[i] = (uint8_t)lds_u8(pk, pbase + (uint32_t)p);
        }
    }
}

// Four LDS bytes at rb + o.{x,y,z,w}, as one little-endian word.
__device__ __forceinline__ uint32_t lds_gather4(const uint8_t *lds, uint32_t rb, const uint4 &o)
{
    uint32_t b0 = lds[rb + o.x], b1 = lds[rb + o.y], b2 = lds[rb + o.z], b3 = lds[rb + o.w];
    return b0 | b1 << 8 | b2 << 16 | b3 << 24;
}

// Pack chunks [c0, c1) of A with the chunk table: one division per chunk
// finds the record and phase of its first byte, the table entry of that
// phase gives the 16 typed offsets, and the bytes are gathered from the
// staged span.  Only the two edge chunks of a transfer go byte by byte.
__device__ __forceinline__ void dense_pack_tile_c(const DevLayout &L, const XferArgs &A, int64_t c0, int64_t c1,
                                                  uint8_t *lds)
{
    const DevRecords &R = L.rec;
    const int64_t P_lo = max(16 * c0 - A.head, (int64_t)0);
    const int64_t P_hi = min(16 * c1 - A.head, A.nbytes);
    const uint64_t s_lo = (uint64_t)(A.off + P_lo);
    const uint64_t e0 = magic_div(s_lo, R.dU);
    const uint64_t e1 = magic_div((uint64_t)(A.off + P_hi - 1), R.dU);
    const int64_t t_lo = R.B0 + (int64_t)e0 * R.X + R.lo;
    const int64_t t_hi = R.B0 + (int64_t)e1 * R.X + R.hi;
    const uint32_t U = (uint32_t)R.U, X = (uint32_t)R.X;
    uint32_t *tab = (uint32_t *)lds;
    uint8_t *span = lds + 64 * U;
    for (uint32_t i = threadIdx.x; i < 4 * U; i += blockDim.x) ((uint4 *)tab)[i] = gld((const uint4 *)R.ctab, i);
    const uint32_t base = stage_span(span, A.typed + t_lo, A.typed + t_hi);
    __syncthreads();
    const uint32_t q0 = (uint32_t)(s_lo - e0 * (uint64_t)U);  // phase of s_lo in record e0
    const int32_t r00 = (int32_t)(16 * c0 - A.head - P_lo);   // chunk c0's start, from P_lo (-15 .. 0)
    const int32_t npk = (int32_t)(P_hi - P_lo);
    uint8_t *const out = A.packed - A.head + 16 * c0;
    const uint32_t nc = (uint32_t)(c1 - c0);
    for (uint32_t k = threadIdx.x; k < nc; k += blockDim.x) {
        const int32_t pr = r00 + 16 * (int32_t)k;
        if (pr >= 0 && pr + 16 <= npk) {
            const uint32_t rel = (uint32_t)pr + q0;
            const uint32_t er = magic_div32(rel, R.dU32);
            const uint32_t q = rel - er * U;
            const uint32_t rb = base + er * X;
            const uint4 *e = (const uint4 *)(tab + 16 * q);
            const uint4 o0 = e[0], o1 = e[1], o2 = e[2], o3 = e[3];
            u32x4 v = {lds_gather4(span, rb, o0), lds_gather4(span, rb, o1), lds_gather4(span, rb, o2),
                       lds_gather4(span, rb, o3)};
            store_out(A, (out + 16 * k), v);
        } else {
            const int32_t a = pr > 0 ? pr : 0, b = pr + 16 < npk ? pr + 16 : npk;
            for (int32_t i = a; i < b; i++) {
                const uint32_t rel = (uint32_t)i + q0;
                const uint32_t er = magic_div32(rel, R.dU32);
                const uint32_t q = rel - er * U;
                gptr(out)[16 * k + (uint32_t)(i - pr)] = span[base + er * X + tab[16 * q]];
            }
        }
    }
}

// Unpack chunks [c0, c1) of A with the dword table.  The LDS window holds
// the packed bytes of records e0 - 1 .. e1 + 1 (clipped to the transfer), so
// every typed dword that overlaps this tile's records can be assembled
// whole: a dword shared with a neighbouring tile is written by both with the
// same bytes.  Away from the transfer's ends nothing is clipped and no byte
// needs a range test; gap bytes are never written.
__device__ __forceinline__ void dense_unpack_tile_d(const DevLayout &L, const XferArgs &A, int64_t c0, int64_t c1,
                                                    uint8_t *lds)
{
    const DevRecords &R = L.rec;
    const int64_t P_lo = max(16 * c0 - A.head, (int64_t)0);
    const int64_t P_hi = min(16 * c1 - A.head, A.nbytes);
    const uint64_t e0 = magic_div((uint64_t)(A.off + P_lo), R.dU);
    const uint64_t e1 = magic_div((uint64_t)(A.off + P_hi - 1), R.dU);
    const int64_t t_lo = R.B0 + (int64_t)e0 * R.X + R.lo;
    const int64_t t_hi = R.B0 + (int64_t)e1 * R.X + R.hi;
    const uint32_t U = (uint32_t)R.U, X = (uint32_t)R.X;
    // window [W0, W1) in transfer-relative packed positions, and its clip
    const int64_t W0 = ((int64_t)e0 - 1) * U - A.off;
    const int64_t W1 = ((int64_t)e1 + 2) * U - A.off;
    const int64_t Wc0 = W0 > 0 ? W0 : 0, Wc1 = W1 < A.nbytes ? W1 : A.nbytes;
    const bool clipped = Wc0 != W0 || Wc1 != W1;
    uint32_t *tab = (uint32_t *)lds;
    uint8_t *pk = lds + 16 * X;
    for (uint32_t i = threadIdx.x; i < X; i += blockDim.x) ((uint4 *)tab)[i] = gld((const uint4 *)R.dtab, i);
    const uint32_t pbase = stage_span(pk, A.packed + Wc0, A.packed + Wc1);
    __syncthreads();
    // window position w (from W0) sits at LDS offset pbase + w - (Wc0 - W0);
    // positions in [vlo, vhi) were staged
    const uint32_t vlo = (uint32_t)(Wc0 - W0), vhi = (uint32_t)(Wc1 - W0);
    uint8_t *t0 = const_cast<uint8_t *>(A.typed) + t_lo;  // typed byte of (record e0, offset lo)
    const uintptr_t d_lo = (uintptr_t)t0 & ~(uintptr_t)3;
    const uint32_t skew = (uint32_t)((uintptr_t)t0 - d_lo);
    const uint32_t tspan = (uint32_t)(t_hi - t_lo);
    const uint32_t ndw = (skew + tspan + 3) >> 2;
    for (uint32_t j = threadIdx.x; j < ndw; j += blockDim.x) {
        // typed offset of the dword from record e0 - 1's lo
        const uint32_t r = 4 * j - skew + X;
        const uint32_t er = magic_div32(r, R.dX32);
        const uint32_t d = r - er * X;
        const uint4 e = ((const uint4 *)tab)[d];
        const uint32_t wb = er * U;  // window position of record e0 - 1 + er
        uint32_t w0 = wb + (e.x & 0xffffu), w1 = wb + (e.x >> 16), w2 = wb + (e.y & 0xffffu), w3 = wb + (e.y >> 16);
        uint32_t m = e.z;
        if (clipped) {
            m &= (w0 - vlo < vhi - vlo ? 1u : 0u) | (w1 - vlo < vhi - vlo ? 2u : 0u) |
                 (w2 - vlo < vhi - vlo ? 4u : 0u) | (w3 - vlo < vhi - vlo ? 8u : 0u);
            w0 = (m & 1u) ? w0 : vlo;
            w1 = (m & 2u) ? w1 : vlo;
            w2 = (m & 4u) ? w2 : vlo;
            w3 = (m & 8u) ? w3 : vlo;
        }
        if (!m) continue;
        const uint32_t sh = pbase - vlo;
        const uint32_t v = lds_gather4(pk, sh, uint4{w0, w1, w2, w3});
        uint8_t *D = (uint8_t *)(d_lo + 4 * (uintptr_t)j);
        if (m == 15u) {
            *gptr((uint32_t *)D) = v;
        } else {
            do {
                const int i = __builtin_ctz(m);
                gptr(D)[i] = (uint8_t)(v >> (8 * i));
                m &= m - 1;
            } while (m);
        }
    }
}

__device__ __forceinline__ void dense_pack_tile(const DevLayout &L, const XferArgs &A, int64_t c0, int64_t c1,
                                                uint8_t *lds)
{
    if (L.rec.ctab) dense_pack_tile_c(L, A, c0, c1, lds);
    else dense_pack_tile_b(L, A, c0, c1, lds);
}

__device__ __forceinline__ void dense_unpack_tile(const DevLayout &L, const XferArgs &A, int64_t c0, int64_t c1,
                                                  uint8_t *lds)
{
    if (L.rec.dtab) dense_unpack_tile_d(L, A, c0, c1, lds);
    else dense_unpack_tile_b(L, A, c0, c1, lds);
}

}  // namespace mdt

namespace mdt {

// ---------------------------------------------------------------------------
// run tables (every group one run, e.g. hindexed of bytes): a workgroup
// caches its tile's slice of the group prefix and displacement tables in LDS
// so each lane finds its run by an LDS binary search instead of a chain of
// dependent global loads.

constexpr int RUNS_CACHE = 2048;

struct RunsCache {
    int64_t pre[RUNS_CACHE + 1];
    int64_t disp[RUNS_CACHE];
};

// Load groups covering stream bytes [s_lo, s_hi) of one element into C.
// Returns the number of cached groups, or -1 when the tile does not fit
// (several elements, or more groups than the cache holds).
__device__ __forceinline__ int64_t runs_cache_fill(const DevLayout &L, const XferArgs &A, uint64_t s_lo, uint64_t s_hi,
                                                   RunsCache &C, int64_t &g0, uint64_t &ebase, int64_t &eaddr)
{
    uint64_t e0 = A.elem1 ? 0 : magic_div(s_lo, L.dsize);
    uint64_t e1 = A.elem1 ? 0 : magic_div(s_hi - 1, L.dsize);
    if (e0 != e1) return -1;
    ebase = e0 * (uint64_t)L.size;
    eaddr = (int64_t)e0 * L.extent;
    g0 = find_group(L, s_lo - ebase);
    int64_t g1 = find_group(L, s_hi - 1 - ebase);
    int64_t n = g1 - g0 + 1;
    if (n > RUNS_CACHE) return -1;
    for (int64_t i = threadIdx.x; i <= n; i += blockDim.x) C.pre[i] = gld(L.gpre, g0 + i);
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) C.disp[i] = gld(L.gdisp, g0 + i);
    __syncthreads();
    return n;
}

// cached group holding element-relative position q
__device__ __forceinline__ int runs_find(const RunsCache &C, int n, uint64_t q)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if ((uint64_t)C.pre[mid] <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Chunk c of the tile lies whole inside the transfer's range.
__device__ __forceinline__ bool runs_whole(const XferArgs &A, int64_t c, int64_t cend)
{
    const int64_t lo = 16 * c - A.head;
    return c < cend && lo >= 0 && lo + 16 <= A.nbytes;
}

// Unpack: scatter a whole chunk, already loaded, run by run.
__device__ __forceinline__ void runs_scatter(const XferArgs &A, const RunsCache &C, int n, uint64_t ebase,
                                             int64_t eaddr, int64_t c, const V4 &acc)
{
    uint64_t q = (uint64_t)(A.off + 16 * c - A.head) - ebase;
    int i = runs_find(C, n, q);
    uint8_t *typed = const_cast<uint8_t *>(A.typed);
    int k = 0;
    while (k < 16 && i < n) {
        const int64_t rem = C.pre[i + 1] - (int64_t)q;
        const int take = rem < 16 - k ? (int)rem : 16 - k;
        if (take > 0) scatter(acc, k, typed + eaddr + C.disp[i] + ((int64_t)q - C.pre[i]), take);
        q += take;
        k += take;
        i++;
    }
}

// Any chunk of the tile (clipped by the transfer's range, or spread over
// more runs than the fast paths take), one run at a time.
template <bool UNPACK>
__device__ __forceinline__ void runs_chunk(const XferArgs &A, const RunsCache &C, int n, uint64_t ebase, int64_t eaddr,
                                           int64_t c)
{
    const uint8_t *typed = A.typed;
    const int64_t lo = 16 * c - A.head;
    const int64_t a = lo > 0 ? lo : 0;
    const int64_t b = lo + 16 < A.nbytes ? lo + 16 : A.nbytes;
    int k = (int)(a - lo), m = (int)(b - a);
    uint64_t q = (uint64_t)(A.off + a) - ebase;
    int i = runs_find(C, n, q);
    V4 acc = {0u, 0u, 0u, 0u};
    if (UNPACK) {
        u32x4 v = __builtin_nontemporal_load(gptr((const u32x4 *)(A.packed - A.head + 16 * c)));
        acc = V4{v.x, v.y, v.z, v.w};
    }
    while (m > 0 && i < n) {
        int64_t in = (int64_t)q - C.pre[i];
        int64_t rem = C.pre[i + 1] - (int64_t)q;
        int take = rem < m ? (int)rem : m;
        const int64_t addr = eaddr + C.disp[i] + in;
        if (UNPACK) {
            scatter(acc, k, const_cast<uint8_t *>(typed) + addr, take);
        } else {
            if (take == 16) acc = load16_any(typed + addr);
            else gather_piece(acc, k, typed + addr, take);
        }
        q += take;
        k += take;
        m -= take;
        i++;
    }
    if (!UNPACK) {
        uint8_t *dst = A.packed - A.head + 16 * c;
        if (a == lo && b == lo + 16) {
            u32x4 v = {acc.w0, acc.w1, acc.w2, acc.w3};
            store_out(A, dst, v);
        } else {
            for (int j = (int)(a - lo); j < (int)(b - lo); j++) gptr(dst)[j] = (uint8_t)byte_at(acc, j);
        }
    }
}

template <bool UNPACK>
__device__ __forceinline__ void runs_tile(const DevLayout &L, const XferArgs &A, int64_t c0, int64_t c1, RunsCache &C)
{
    const int64_t P_lo = max(16 * c0 - A.head, (int64_t)0);
    const int64_t P_hi = min(16 * c1 - A.head, A.nbytes);
    int64_t g0;
    uint64_t ebase;
    int64_t eaddr;
    int64_t n = runs_cache_fill(L, A, (uint64_t)(A.off + P_lo), (uint64_t)(A.off + P_hi), C, g0, ebase, eaddr);
    if (n < 0) {
        if (UNPACK) {
            for (int64_t s0 = c0; s0 < c1; s0 += 1024) unpack_tile4<KIND_MULTI>(L, A, s0, min(s0 + 1024, c1));
        } else {
            for (int64_t s0 = c0; s0 < c1; s0 += 1024) pack_tile4<KIND_MULTI>(L, A, s0, min(s0 + 1024, c1));
        }
        return;
    }
    const int nc = (int)n;
    if (!UNPACK) {
        // pack gathers one chunk at a time: issuing all four chunks' gathers
        // together measured slower (many small loads per chunk)
        for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) runs_chunk<false>(A, C, nc, ebase, eaddr, c);
        return;
    }
    // unpack: a lane's chunks c + 256k (k < 4) per 1024-chunk step, packed
    // loads first (stores do not wait)
    for (int64_t s0 = c0; s0 < c1; s0 += 1024) {
        const int64_t c = s0 + threadIdx.x;
        const int64_t cend = min(s0 + 1024, c1);
        V4 a0 = {0u, 0u, 0u, 0u}, a1 = a0, a2 = a0, a3 = a0;
        uint32_t fast = 0;
        if (runs_whole(A, c, cend)) {
            u32x4 v = __builtin_nontemporal_load(gptr((const u32x4 *)(A.packed - A.head + 16 * c)));
            a0 = V4{v.x, v.y, v.z, v.w};
            fast |= 1u;
        }
        if (runs_whole(A, c + 256, cend)) {
            u32x4 v = __builtin_nontemporal_load(gptr((const u32x4 *)(A.packed - A.head + 16 * (c + 256))));
            a1 = V4{v.x, v.y, v.z, v.w};
            fast |= 2u;
        }
        if (runs_whole(A, c + 512, cend)) {
            u32x4 v = __builtin_nontemporal_load(gptr((const u32x4 *)(A.packed - A.head + 16 * (c + 512))));
            a2 = V4{v.x, v.y, v.z, v.w};
            fast |= 4u;
        }
        if (runs_whole(A, c + 768, cend)) {
            u32x4 v = __builtin_nontemporal_load(gptr((const u32x4 *)(A.packed - A.head + 16 * (c + 768))));
            a3 = V4{v.x, v.y, v.z, v.w};
            fast |= 8u;
        }
        if (fast & 1u) runs_scatter(A, C, nc, ebase, eaddr, c, a0);
        if (fast & 2u) runs_scatter(A, C, nc, ebase, eaddr, c + 256, a1);
        if (fast & 4u) runs_scatter(A, C, nc, ebase, eaddr, c + 512, a2);
        if (fast & 8u) runs_scatter(A, C, nc, ebase, eaddr, c + 768, a3);
#pragma unroll 1
        for (int k = 0; k < 4; k++) {
            const int64_t ck = c + 256 * k;
            if (ck < cend && !((fast >> k) & 1u)) runs_chunk<true>(A, C, nc, ebase, eaddr, ck);
        }
    }
}

}  // namespace mdt
