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
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "core.h"
#include "device.h"
#include "xfer.h"

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

int device_tables_resident(Compiled *c, DeviceTables **out)
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
    return MDT_ERR_STATE;
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
    size_t off_ptab = off; off += al256(c->rec_ptab.size() * sizeof(uint32_t));
    size_t off_ttab = off; off += al256(c->rec_ttab.size() * sizeof(uint32_t));
    size_t off_ctab = off; off += al256(c->rec_ctab.size() * sizeof(uint32_t));
    size_t off_dtab = off; off += al256(c->rec_dtab.size() * sizeof(uint32_t));
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
    put(off_ptab, c->rec_ptab.data(), c->rec_ptab.size() * 4);
    put(off_ttab, c->rec_ttab.data(), c->rec_ttab.size() * 4);
    put(off_ctab, c->rec_ctab.data(), c->rec_ctab.size() * 4);
    put(off_dtab, c->rec_dtab.data(), c->rec_dtab.size() * 4);
    DevLayout &L = d->lay;
    if (nsh) L.shape0 = shapes[0];
    L.shapes = nsh ? (const DevShape *)(base + off_shapes) : nullptr;
    L.gdisp = H.gdisp ? (const int64_t *)(base + off_gdisp) : nullptr;
    L.gpre = H.gpre ? (const int64_t *)(base + off_gpre) : nullptr;
    L.grpre = H.grpre ? (const int64_t *)(base + off_grpre) : nullptr;
    L.gshape = H.gshape ? (const int32_t *)(base + off_gshape) : nullptr;
    L.gdir = H.gdir ? (const int32_t *)(base + off_gdir) : nullptr;
    L.rec.ptab = H.rec.ptab ? (const uint32_t *)(base + off_ptab) : nullptr;
    L.rec.ttab = H.rec.ttab ? (const uint32_t *)(base + off_ttab) : nullptr;
    L.rec.ctab = H.rec.ctab ? (const uint32_t *)(base + off_ctab) : nullptr;
    L.rec.dtab = H.rec.dtab ? (const uint32_t *)(base + off_dtab) : nullptr;
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

// Workgroup b takes tiles b, b + grid, ... (normally grid = tiles).
template <int KIND, bool UNPACK>
__global__ __launch_bounds__(256) void xfer_kernel(const DevLayout L, const XferArgs A)
{
    const int64_t ntiles = (A.nchunks + A.tile_chunks - 1) / A.tile_chunks;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int64_t c0 = t * A.tile_chunks;
        int64_t cend = c0 + A.tile_chunks < A.nchunks ? c0 + A.tile_chunks : A.nchunks;
        // tile_chunks <= 1024: at most four chunks per lane
        if (UNPACK) unpack_tile4<KIND>(L, A, c0, cend);
        else pack_tile4<KIND>(L, A, c0, cend);
    }
}

// typed copy: one tile of 1024 chunks per workgroup (four per lane)
template <int KS, int KD>
__global__ __launch_bounds__(256) void copy_kernel(const DevLayout Ls, const DevLayout Ld, const CopyArgs A)
{
    const int64_t ntiles = (A.nchunks + 1023) / 1024;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t c0 = t * 1024;
        const int64_t cend = c0 + 1024 < A.nchunks ? c0 + 1024 : A.nchunks;
        copy_tile4<KS, KD>(Ls, Ld, A, c0, cend);
    }
}

// dense record streams: one tile of chunks per workgroup, staged in LDS
template <bool UNPACK>
__global__ __launch_bounds__(256) void dense_kernel(const DevLayout L, const XferArgs A)
{
    extern __shared__ __align__(16) uint8_t lds_dyn[];
    const int64_t ntiles = (A.nchunks + A.tile_chunks - 1) / A.tile_chunks;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int64_t c0 = t * A.tile_chunks;
        int64_t c1 = c0 + A.tile_chunks < A.nchunks ? c0 + A.tile_chunks : A.nchunks;
        if (UNPACK) dense_unpack_tile(L, A, c0, c1, lds_dyn);
        else dense_pack_tile(L, A, c0, c1, lds_dyn);
        __syncthreads();  // LDS is reused by the next tile
    }
}

// run tables: tile of chunks with the tile's groups cached in LDS
template <bool UNPACK>
__global__ __launch_bounds__(256) void runs_kernel(const DevLayout L, const XferArgs A)
{
    __shared__ RunsCache cache;
    const int64_t ntiles = (A.nchunks + A.tile_chunks - 1) / A.tile_chunks;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int64_t c0 = t * A.tile_chunks;
        int64_t c1 = c0 + A.tile_chunks < A.nchunks ? c0 + A.tile_chunks : A.nchunks;
        runs_tile<UNPACK>(L, A, c0, c1, cache);
        __syncthreads();  // the cache is refilled for the next tile
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

// flatten over count consecutive elements: lane i writes segment off + i of
// the count form (the element's segments repeated at multiples of the
// extent; with `merge`, each element's last segment joined to the next
// element's first).  TABLE: segments come from the merged-segment table,
// else from the layout's runs.
template <bool TABLE>
__global__ __launch_bounds__(256) void flatten_count_kernel(const DevLayout L, const mdt_iov *segs, int64_t n,
                                                            int merge, int64_t count, int64_t extent, int64_t off,
                                                            int64_t m, mdt_iov *out, uintptr_t base)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const int64_t g = off + i;
    auto seg = [&](int64_t j, int64_t *a, int64_t *l) {
        if (TABLE) {
            mdt_iov v = segs[j];
            *a = (int64_t)(intptr_t)v.iov_base;
            *l = v.iov_len;
        } else {
            RunInfo r = run_at(L, (uint64_t)j);
            *a = r.addr;
            *l = r.len;
        }
    };
    int64_t a, l;
    if (!merge) {
        const int64_t q = g / n;
        seg(g - q * n, &a, &l);
        a += q * extent;
    } else if (n == 1) {
        seg(0, &a, &l);
        l *= count;
    } else if (g == 0) {
        seg(0, &a, &l);
    } else {
        const int64_t q = (g - 1) / (n - 1), j = (g - 1) - q * (n - 1) + 1;
        seg(j, &a, &l);
        a += q * extent;
        if (j == n - 1 && q < count - 1) {
            int64_t a0, l0;
            seg(0, &a0, &l0);
            l += l0;
        }
    }
    out[i].iov_base = (void *)(base + (uintptr_t)a);
    out[i].iov_len = l;
}

// ---------------------------------------------------------------------------
// launch

// Workgroups of a launch: one per tile by default (measured faster than a
// grid capped at the resident capacity, whose second round of workgroups
// runs as a serialized tail); MDT_WG_PER_CU > 0 caps it for experiments.
static int64_t launch_grid(int64_t ntiles)
{
    static const int64_t cap = [] {
        const char *e = getenv("MDT_WG_PER_CU");
        int per_cu = e && *e ? atoi(e) : 0;
        if (per_cu <= 0) return (int64_t)0;
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        return (int64_t)n * per_cu;
    }();
    return cap > 0 && ntiles > cap ? cap : ntiles;
}

int64_t default_tile_chunks(int64_t nchunks)
{
    // 4 chunks per lane for large transfers, 1 for small ones (MDT_CHUNK_TILE
    // = 64..1024 fixes it, for tuning)
    static const int64_t fixed = [] {
        const char *e = getenv("MDT_CHUNK_TILE");
        int v = e && *e ? atoi(e) : 0;
        return (int64_t)(v == 64 || v == 128 || v == 256 || v == 512 || v == 1024 ? v : 0);
    }();
    if (fixed) return fixed;
    return nchunks >= ((int64_t)1 << 19) ? 1024 : 256;
}

static bool dense_enabled()
{
    static const bool on = [] {
        const char *e = getenv("MDT_DENSE");
        return !(e && e[0] == '0');
    }();
    return on;
}

static bool runs_enabled()
{
    static const bool on = [] {
        const char *e = getenv("MDT_RUNS_CACHE");
        return !(e && e[0] == '0');
    }();
    return on;
}

bool use_dense(const DevLayout &L, const XferArgs &A, bool unpack)
{
    const DevRecords &R = L.rec;
    if (!R.on || !dense_enabled()) return false;
    if (R.count1_only && A.off + A.nbytes > L.size) return false;
    return !unpack || R.unpack_ok;
}

bool use_runs(const DevLayout &L) { return L.kind == KIND_MULTI && L.runs_only && runs_enabled(); }

int launch_xfer(const DevLayout &L, const XferArgs &A0, bool unpack, hipStream_t s)
{
    if (A0.nbytes == 0 || L.kind == KIND_EMPTY) return MDT_SUCCESS;
    XferArgs A = A0;
    A.elem1 = A.off + A.nbytes <= L.size;
    A.keep = !unpack && A.nbytes <= KEEP_PACKED_MAX;
    if (use_dense(L, A, unpack)) {
        A.tile_chunks = L.rec.tile_chunks;
        int64_t grid = launch_grid((A.nchunks + A.tile_chunks - 1) / A.tile_chunks);
        size_t lds = (size_t)L.rec.lds_bytes;
        if (unpack) hipLaunchKernelGGL(dense_kernel<true>, dim3((unsigned)grid), dim3(256), lds, s, L, A);
        else hipLaunchKernelGGL(dense_kernel<false>, dim3((unsigned)grid), dim3(256), lds, s, L, A);
        HIPCHK(hipGetLastError());
        return MDT_SUCCESS;
    }
    if (use_runs(L)) {
        A.tile_chunks = 1024;
        int64_t grid = launch_grid((A.nchunks + A.tile_chunks - 1) / A.tile_chunks);
        if (unpack) hipLaunchKernelGGL(runs_kernel<true>, dim3((unsigned)grid), dim3(256), 0, s, L, A);
        else hipLaunchKernelGGL(runs_kernel<false>, dim3((unsigned)grid), dim3(256), 0, s, L, A);
        HIPCHK(hipGetLastError());
        return MDT_SUCCESS;
    }
    if (A.tile_chunks <= 0 || A.tile_chunks > 1024) A.tile_chunks = default_tile_chunks(A.nchunks);
    int64_t grid = launch_grid((A.nchunks + A.tile_chunks - 1) / A.tile_chunks);
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

template <int KS>
static void launch_copy_kd(const DevLayout &Ls, const DevLayout &Ld, const CopyArgs &A, dim3 g, hipStream_t s)
{
    if (Ld.kind == KIND_CONTIG) hipLaunchKernelGGL((copy_kernel<KS, KIND_CONTIG>), g, dim3(256), 0, s, Ls, Ld, A);
    else if (Ld.kind == KIND_SINGLE) hipLaunchKernelGGL((copy_kernel<KS, KIND_SINGLE>), g, dim3(256), 0, s, Ls, Ld, A);
    else hipLaunchKernelGGL((copy_kernel<KS, KIND_MULTI>), g, dim3(256), 0, s, Ls, Ld, A);
}

int launch_copy(const DevLayout &Ls, const DevLayout &Ld, const CopyArgs &A, hipStream_t s)
{
    if (A.nbytes == 0 || Ls.kind == KIND_EMPTY || Ld.kind == KIND_EMPTY) return MDT_SUCCESS;
    const dim3 g((unsigned)launch_grid((A.nchunks + 1023) / 1024));
    if (Ls.kind == KIND_CONTIG) launch_copy_kd<KIND_CONTIG>(Ls, Ld, A, g, s);
    else if (Ls.kind == KIND_SINGLE) launch_copy_kd<KIND_SINGLE>(Ls, Ld, A, g, s);
    else launch_copy_kd<KIND_MULTI>(Ls, Ld, A, g, s);
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
    A.elem1 = 0;
    return A;
}

int launch_flatten(Compiled *c, DeviceTables *d, int64_t off, int64_t m, mdt_iov *out, const void *base,
                   hipStream_t s, const SegCount *sc)
{
    if (m <= 0) return MDT_SUCCESS;
    if ((m + 255) / 256 > (int64_t)UINT32_MAX) return MDT_ERR_COUNT;
    dim3 g((unsigned)((m + 255) / 256)), b(256);
    const bool counted = sc && sc->count != 1;
    if (c->merge_free) {
        if (counted)
            hipLaunchKernelGGL(flatten_count_kernel<false>, g, b, 0, s, d->lay, (const mdt_iov *)nullptr, sc->n,
                               (int)sc->merge, sc->count, sc->extent, off, m, out, (uintptr_t)base);
        else
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
        if (counted)
            hipLaunchKernelGGL(flatten_count_kernel<true>, g, b, 0, s, d->lay, (const mdt_iov *)d->d_segs, sc->n,
                               (int)sc->merge, sc->count, sc->extent, off, m, out, (uintptr_t)base);
        else
            hipLaunchKernelGGL(flatten_table_kernel, g, b, 0, s, d->d_segs, off, m, out, (uintptr_t)base);
    }
    HIPCHK(hipGetLastError());
    return MDT_SUCCESS;
}

}  // namespace mdt

extern "C" MDT_API int mdt_last_hip_error(void) { return mdt::g_last_hip; }
