// device.hip -- gfx950 kernels for pack / unpack / flatten and their launch
// paths, plus the resident device tables of committed types.
//
// Pack (gather) and unpack (scatter) are pure data movement, bound by HBM
// bandwidth; there is no arithmetic to put on matrix cores.  The packed
// side is always touched as aligned 16-byte chunks (one dwordx4 per lane,
// coalesced across the wavefront); the typed side is touched at whatever
// byte alignment the layout dictates, realigned in registers with
// v_alignbyte so that every memory access is naturally aligned:
//   - each lane owns one 16-byte chunk of the packed stream at a time and
//     locates its first byte in the layout program (magic divisions down the
//     loop nest, directory-guided search over a group table);
//   - it then walks the runs that cover its 16 bytes (usually one, at most a
//     few for tiny blocks), gathering from / scattering to the typed buffer;
//   - a chunk whose bytes all lie in one run takes a straight 16-byte path;
//     otherwise bytes are merged dword by dword.
// Unpack writes a byte only if the typemap covers it (gaps are untouched)
// and each byte is written by the lane that owns its packed chunk, so
// neighbouring lanes never race.  Work is split in tiles of consecutive
// chunks per workgroup, and tiles are dealt so that each XCD (own L2) gets a
// contiguous range of the stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "core.h"
#include "device.h"

namespace mdt {

static thread_local int g_last_hip = 0;
void set_hip_error(int e) { g_last_hip = e; }

#define HIPCHK(x)                         \
    do {                                  \
        hipError_t e_ = (x);              \
        if (e_ != hipSuccess) {           \
            set_hip_error((int)e_);       \
            return MDT_ERR_HIP;           \
        }                                 \
    } while (0)

// ---------------------------------------------------------------------------
// resident tables

static size_t al256(size_t n) { return (n + 255) & ~(size_t)255; }

void free_device_tables(DeviceTables *d)
{
    if (!d) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (d->device >= 0 && cur != d->device) (void)hipSetDevice(d->device);
    for (void *p : d->allocs) (void)hipFree(p);
    d->allocs.clear();
    if (d->device >= 0 && cur >= 0 && cur != d->device) (void)hipSetDevice(cur);
}

int device_tables(Compiled *c, DeviceTables **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0) {
        set_hip_error((int)e);
        return MDT_ERR_HIP;
    }
    std::lock_guard<std::mutex> g(c->dev_mu);
    if ((size_t)dev < c->dev.size() && c->dev[dev]) {
        *out = c->dev[dev].get();
        return MDT_SUCCESS;
    }
    auto d = std::make_unique<DeviceTables>();
    d->device = dev;
    d->lay = c->host;
    const DevLayout &H = c->host;
    // one blob: shapes, leaf arrays, group arrays, directory, descriptor
    size_t nsh = c->shapes.size();
    size_t off_shapes = 0;
    size_t off = al256(nsh * sizeof(DevShape));
    std::vector<size_t> leaf_off;
    for (auto &v : c->leaf_store) {
        leaf_off.push_back(off);
        off += al256(v.size() * sizeof(int64_t));
    }
    size_t off_gdisp = off; off += al256(c->gdisp.size() * sizeof(int64_t));
    size_t off_gpre = off; off += al256(c->gpre.size() * sizeof(int64_t));
    size_t off_grpre = off; off += al256(c->grpre.size() * sizeof(int64_t));
    size_t off_gshape = off; off += al256(c->gshape.size() * sizeof(int32_t));
    size_t off_gdir = off; off += al256(c->gdir.size() * sizeof(int32_t));
    size_t off_lay = off; off += al256(sizeof(DevLayout));
    std::vector<uint8_t> blob(off, 0);
    uint8_t *base = nullptr;
    e = hipMalloc((void **)&base, off);
    if (e != hipSuccess) {
        set_hip_error((int)e);
        return e == hipErrorOutOfMemory ? MDT_ERR_NO_MEM : MDT_ERR_HIP;
    }
    d->allocs.push_back(base);
    // shapes with device leaf pointers
    std::vector<DevShape> shapes = c->shapes;
    size_t k = 0;
    for (DevShape &S : shapes) {
        if (S.nleaf > LEAFI) {
            const int64_t *p = (const int64_t *)(base + leaf_off[k]);
            size_t n = (size_t)S.nleaf;
            S.loff_p = p;
            S.llen_p = p + n;
            S.lpre_p = p + 2 * n;
            std::memcpy(blob.data() + leaf_off[k], c->leaf_store[k].data(), c->leaf_store[k].size() * 8);
            k++;
        }
    }
    if (nsh) std::memcpy(blob.data() + off_shapes, shapes.data(), nsh * sizeof(DevShape));
    auto put = [&](size_t o, const void *src, size_t n) {
        if (n) std::memcpy(blob.data() + o, src, n);
    };
    put(off_gdisp, c->gdisp.data(), c->gdisp.size() * 8);
    put(off_gpre, c->gpre.data(), c->gpre.size() * 8);
    put(off_grpre, c->grpre.data(), c->grpre.size() * 8);
    put(off_gshape, c->gshape.data(), c->gshape.size() * 4);
    put(off_gdir, c->gdir.data(), c->gdir.size() * 4);
    DevLayout &L = d->lay;
    if (nsh) L.shape0 = shapes[0];
    L.shapes = nsh ? (const DevShape *)(base + off_shapes) : nullptr;
    L.gdisp = H.gdisp ? (const int64_t *)(base + off_gdisp) : nullptr;
    L.gpre = H.gpre ? (const int64_t *)(base + off_gpre) : nullptr;
    L.grpre = H.grpre ? (const int64_t *)(base + off_grpre) : nullptr;
    L.gshape = H.gshape ? (const int32_t *)(base + off_gshape) : nullptr;
    L.gdir = H.gdir ? (const int32_t *)(base + off_gdir) : nullptr;
    std::memcpy(blob.data() + off_lay, &L, sizeof(DevLayout));
    d->d_lay = (DevLayout *)(base + off_lay);
    e = hipMemcpy(base, blob.data(), off, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        set_hip_error((int)e);
        free_device_tables(d.get());
        return MDT_ERR_HIP;
    }
    if (c->dev.size() <= (size_t)dev) c->dev.resize(dev + 1);
    c->dev[dev] = std::move(d);
    *out = c->dev[dev].get();
    return MDT_SUCCESS;
}

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

template <int KIND, bool UNPACK>
__global__ __launch_bounds__(256) void xfer_kernel(const DevLayout L, const XferArgs A)
{
    int64_t c0 = xcd_tile() * A.tile_chunks;
    int64_t cend = c0 + A.tile_chunks < A.nchunks ? c0 + A.tile_chunks : A.nchunks;
    for (int64_t c = c0 + threadIdx.x; c < cend; c += 256) {
        if (UNPACK) unpack_chunk<KIND>(L, A, c);
        else pack_chunk<KIND>(L, A, c);
    }
}

// flatten: one lane per segment
__global__ __launch_bounds__(256) void flatten_kernel(const DevLayout L, int64_t off, int64_t m, mdt_iov *out,
                                                     uintptr_t base)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    RunInfo r = run_at(L, (uint64_t)(off + i));
    out[i].iov_base = (void *)(base + (uintptr_t)r.addr);
    out[i].iov_len = r.len;
}

__global__ __launch_bounds__(256) void flatten_table_kernel(const mdt_iov *segs, int64_t off, int64_t m,
                                                           mdt_iov *out, uintptr_t base)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    mdt_iov s = segs[off + i];
    out[i].iov_base = (void *)(base + (uintptr_t)s.iov_base);
    out[i].iov_len = s.iov_len;
}

// ---------------------------------------------------------------------------
// launch

int64_t default_tile_chunks(int64_t nchunks)
{
    // 4 chunks per lane for large transfers, 1 for small ones
    return nchunks >= ((int64_t)1 << 19) ? 1024 : 256;
}

int launch_xfer(const DevLayout &L, const XferArgs &A0, bool unpack, hipStream_t s)
{
    if (A0.nbytes == 0 || L.kind == KIND_EMPTY) return MDT_SUCCESS;
    XferArgs A = A0;
    if (A.tile_chunks <= 0) A.tile_chunks = default_tile_chunks(A.nchunks);
    int64_t grid = (A.nchunks + A.tile_chunks - 1) / A.tile_chunks;
    if (grid > 0x7fffffff) return MDT_ERR_ARG;
    dim3 g((unsigned)grid), b(256);
#define LAUNCH(K)                                                                    \
    do {                                                                             \
        if (unpack) hipLaunchKernelGGL((xfer_kernel<K, true>), g, b, 0, s, L, A);    \
        else hipLaunchKernelGGL((xfer_kernel<K, false>), g, b, 0, s, L, A);          \
    } while (0)
    switch (L.kind) {
    case KIND_CONTIG: LAUNCH(KIND_CONTIG); break;
    case KIND_SINGLE: LAUNCH(KIND_SINGLE); break;
    default: LAUNCH(KIND_MULTI); break;
    }
#undef LAUNCH
    HIPCHK(hipGetLastError());
    return MDT_SUCCESS;
}

XferArgs make_args(const void *typed, void *packed, int64_t off, int64_t nbytes)
{
    XferArgs A{};
    A.typed = (const uint8_t *)typed;
    A.packed = (uint8_t *)packed;
    A.off = off;
    A.nbytes = nbytes;
    A.head = (int64_t)((uintptr_t)packed & 15);
    A.nchunks = (A.head + nbytes + 15) / 16;
    A.tile_chunks = 0;
    return A;
}

int launch_flatten(Compiled *c, DeviceTables *d, int64_t off, int64_t m, mdt_iov *out, const void *base,
                   hipStream_t s)
{
    if (m <= 0) return MDT_SUCCESS;
    dim3 g((unsigned)((m + 255) / 256)), b(256);
    if (c->merge_free) {
        hipLaunchKernelGGL(flatten_kernel, g, b, 0, s, d->lay, off, m, out, (uintptr_t)base);
    } else {
        std::lock_guard<std::mutex> lk(c->dev_mu);
        if (!d->d_segs) {
            size_t n = c->seg_addr.size();
            std::vector<mdt_iov> h(n);
            for (size_t i = 0; i < n; i++) {
                h[i].iov_base = (void *)(intptr_t)c->seg_addr[i];
                h[i].iov_len = c->seg_len[i];
            }
            void *p = nullptr;
            HIPCHK(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(mdt_iov)));
            d->allocs.push_back(p);
            HIPCHK(hipMemcpy(p, h.data(), n * sizeof(mdt_iov), hipMemcpyHostToDevice));
            d->d_segs = (mdt_iov *)p;
        }
        hipLaunchKernelGGL(flatten_table_kernel, g, b, 0, s, d->d_segs, off, m, out, (uintptr_t)base);
    }
    HIPCHK(hipGetLastError());
    return MDT_SUCCESS;
}

}  // namespace mdt

extern "C" MDT_API int mdt_last_hip_error(void) { return mdt::g_last_hip; }
