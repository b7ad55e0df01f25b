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

// word i (0..3, 4 reads as 3) of the chunk, by two levels of selects (a
// compare chain would be turned into an indexed stack array)
__device__ __forceinline__ uint32_t sel(const V4 &a, int i)
{
    uint32_t lo = (i & 1) ? a.w1 : a.w0;
    uint32_t hi = (i & 1) ? a.w3 : a.w2;
    return (i & 2) ? hi : (i & 4) ? a.w3 : lo;
}

__device__ __forceinline__ uint32_t byte_at(const V4 &a, int pos)
{
    return (sel(a, pos >> 2) >> (8 * (pos & 3))) & 0xffu;
}

// 4 bytes starting at byte pos (0 <= pos <= 12) of the 16-byte chunk
__device__ __forceinline__ uint32_t dword_at(const V4 &a, int pos)
{
    int w = pos >> 2;
    return __builtin_amdgcn_alignbyte(sel(a, w + 1), sel(a, w), (uint32_t)(pos & 3));
}

// 16 bytes from an arbitrarily aligned source; every dword loaded holds at
// least one of the 16 bytes, so no access leaves the source's pages.
__device__ __forceinline__ V4 load16(const uint8_t *s)
{
    uintptr_t u = (uintptr_t)s;
    V4 r;
    if ((u & 15) == 0) {
        u32x4 v = __builtin_nontemporal_load((const u32x4 *)s);
        r.w0 = v.x; r.w1 = v.y; r.w2 = v.z; r.w3 = v.w;
    } else if ((u & 7) == 0) {
        const u32x2 *p = (const u32x2 *)s;
        u32x2 a = p[0], b = p[1];
        r.w0 = a.x; r.w1 = a.y; r.w2 = b.x; r.w3 = b.y;
    } else if ((u & 3) == 0) {
        const uint32_t *p = (const uint32_t *)s;
        r.w0 = p[0]; r.w1 = p[1]; r.w2 = p[2]; r.w3 = p[3];
    } else {
        const uint32_t *p = (const uint32_t *)(u & ~(uintptr_t)3);
        uint32_t sh = (uint32_t)(u & 3);
        uint32_t d0 = p[0], d1 = p[1], d2 = p[2], d3 = p[3], d4 = p[4];
        r.w0 = __builtin_amdgcn_alignbyte(d1, d0, sh);
        r.w1 = __builtin_amdgcn_alignbyte(d2, d1, sh);
        r.w2 = __builtin_amdgcn_alignbyte(d3, d2, sh);
        r.w3 = __builtin_amdgcn_alignbyte(d4, d3, sh);
    }
    return r;
}

// OR bytes s[0..n) into chunk positions [k, k+n)  (n < 16 or k > 0)
__device__ __forceinline__ void gather_part(V4 &acc, int k, const uint8_t *s, int n)
{
    uint32_t out[4] = {acc.w0, acc.w1, acc.w2, acc.w3};
#pragma unroll
    for (int t = 0; t < 4; t++) {
        int a = max(4 * t, k), b = min(4 * t + 4, k + n);
        if (a < b) {
            uintptr_t u = (uintptr_t)(s + (a - k));
            const uint32_t *p = (const uint32_t *)(u & ~(uintptr_t)3);
            uint32_t sh = (uint32_t)(u & 3);
            int cnt = b - a;
            uint32_t lo = p[0];
            uint32_t hi = ((int)sh + cnt > 4) ? p[1] : 0u;
            uint32_t v = __builtin_amdgcn_alignbyte(hi, lo, sh);
            uint32_t m = cnt >= 4 ? 0xffffffffu : ((1u << (8 * cnt)) - 1u);
            out[t] |= (v & m) << (8 * (a - 4 * t));
        }
    }
    acc.w0 = out[0]; acc.w1 = out[1]; acc.w2 = out[2]; acc.w3 = out[3];
}

// write chunk bytes [k, k+n) to d[0..n): only those bytes are stored
__device__ __forceinline__ void scatter(const V4 &acc, int k, uint8_t *d, int n)
{
    uintptr_t u = (uintptr_t)d;
    if (n == 16) {
        if ((u & 15) == 0) {
            u32x4 v = {acc.w0, acc.w1, acc.w2, acc.w3};
            *(u32x4 *)d = v;
            return;
        }
        if ((u & 7) == 0) {
            u32x2 *p = (u32x2 *)d;
            p[0] = u32x2{acc.w0, acc.w1};
            p[1] = u32x2{acc.w2, acc.w3};
            return;
        }
        if ((u & 3) == 0) {
            uint32_t *p = (uint32_t *)d;
            p[0] = acc.w0; p[1] = acc.w1; p[2] = acc.w2; p[3] = acc.w3;
            return;
        }
    }
    int h = (int)((4 - (u & 3)) & 3);
    if (h > n) h = n;
    for (int i = 0; i < h; i++) d[i] = (uint8_t)byte_at(acc, k + i);
    int j = h;
    for (; j + 4 <= n; j += 4) *(uint32_t *)(d + j) = dword_at(acc, k + j);
    for (; j < n; j++) d[j] = (uint8_t)byte_at(acc, k + j);
}

// ---------------------------------------------------------------------------
// chunk bodies

template <int KIND>
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
    Loc l = locate<KIND>(L, p);
    if (n == 16 && l.rem >= 16) {
        acc = load16(src + l.addr);
    } else {
        for (;;) {
            int take = l.rem < n ? (int)l.rem : n;
            if (take <= 0) break;  // unreachable for a well-formed layout; never spin
            gather_part(acc, k, src + l.addr, take);
            p += take;
            k += take;
            n -= take;
            if (n <= 0) break;
            l = locate<KIND>(L, p);
        }
    }
    uint8_t *dst = A.packed - A.head + 16 * c;
    if (a == lo && b == lo + 16) {
        u32x4 v = {acc.w0, acc.w1, acc.w2, acc.w3};
        __builtin_nontemporal_store(v, (u32x4 *)dst);
    } else {
        for (int i = (int)(a - lo); i < (int)(b - lo); i++) dst[i] = (uint8_t)byte_at(acc, i);
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
    u32x4 v = __builtin_nontemporal_load((const u32x4 *)in);
    V4 acc = {v.x, v.y, v.z, v.w};
    uint64_t p = (uint64_t)(A.off + a);
    uint8_t *dst = const_cast<uint8_t *>(A.typed);
    Loc l = locate<KIND>(L, p);
    for (;;) {
        int take = l.rem < n ? (int)l.rem : n;
        if (take <= 0) break;  // unreachable for a well-formed layout; never spin
        scatter(acc, k, dst + l.addr, take);
        p += take;
        k += take;
        n -= take;
        if (n <= 0) break;
        l = locate<KIND>(L, p);
    }
}

// tile index of this workgroup: the grid is dealt round-robin over the 8
// XCDs, so give XCD x the x-th contiguous share of the tiles
__device__ __forceinline__ int64_t xcd_tile()
{
    int64_t nb = gridDim.x, b = blockIdx.x;
    int64_t q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

}  // namespace mdt
