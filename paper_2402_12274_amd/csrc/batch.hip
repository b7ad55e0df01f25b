// batch.hip -- many pack/unpack requests in one launch per direction.
//
// Launching one kernel per request costs a few microseconds of host and
// dispatch time each; thousands of small requests are then bound by launch
// overhead, not by HBM (MPIX Streams, Background: launch and synchronisation
// cost is a key performance factor).  A batch lowers every request into
// tiles of consecutive 16-byte chunks, lays the request descriptors (pack
// requests first) and the per-request first-tile prefix out in device
// memory, and runs one grid per direction: persistent (workgroups per CU x
// CUs) pulling tiles in a static strided order or from an atomic counter, or
// one workgroup per tile (with or without the tile loop); or it runs each
// request's own single-request kernel.  Tiles run in request order or in the order of the
// typed address they start at (requests that share cache lines then run
// together, neighbours on the same XCD).  Each tile finds its request by
// binary search over the prefix, reads the request's layout program through
// the scalar cache, and runs exactly the tile bodies of the single-request
// kernels, so every byte is identical to the request run alone.  The launch
// can be captured once in a HIP graph and replayed; descriptors are uploaded
// in stream order only when the batch changed.  An autotuner times these
// choices on the batch itself and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include <unistd.h>

#include "core.h"
#include "device.h"
#include "batch_kernel.h"
#include "requests.h"
#include "trace.h"


using namespace mdt;

constexpr uint32_t BATCH_MAGIC = 0x6d647442u;

struct BatchReq {
    TypeNode *type;   // retained
    ReqDesc d;
    int32_t lds;      // dynamic LDS the request's body needs
    TypeNode *type2;  // copy: the destination type (retained), else NULL
    int64_t mean_run; // packed bytes per typed run of the request's type
};

// Tile bodies a request needs its direction's kernel to carry.
int body_bits(const ReqDesc &d) { return d.body | (d.body == BODY_RELAY ? d.pbody | d.ubody : 0); }

// A pack direction whose requests all take the chunk body gathers through
// the caches when some request's runs are shorter than a line: those lines
// hold runs that other tiles (often of other requests) read soon after,
// such as the width-1 and width-4 faces of one side of an array.  Longer
// runs stream.
constexpr int64_t CACHED_RUN_MAX = 127;

int dir_body(int body, int dir, int64_t min_mean_run)
{
    return dir == 0 && body == BODY_CHUNK && min_mean_run <= CACHED_RUN_MAX ? (BODY_CHUNK | BODY_CACHED) : body;
}

// Chunks per tile of a request.  In typed-address order a request of short
// runs gets proportionally shorter tiles (down to a quarter), so that tiles
// of requests whose runs share cache lines -- the width-1 and width-4 faces
// of one side of a halo, 8-byte and 32-byte blocks in the same 128-byte
// lines -- cover the same rows: sorted by typed address they run side by
// side on one XCD and the second access to a line hits its L2.
int64_t tile_chunks_of(const mdt_batch_config &cfg, const BatchReq &r)
{
    const int64_t T = cfg.tile_chunks;
    if (!cfg.order || r.mean_run >= 32) return T;
    const int64_t t = T * std::max<int64_t>(r.mean_run, 8) / 32;
    return std::max<int64_t>(64, t / 64 * 64);
}

struct mdt_batch_s {
    uint32_t magic = BATCH_MAGIC;
    std::vector<BatchReq> reqs;
    mdt_batch_config cfg{1024, 4, 0, 1, 0};
    bool dirty = true;
    uint64_t gen = 0;        // bumped whenever the request list changes
    uint64_t graph_gen = ~0ull;
    int device = -1;
    int ncu = 0;
    // device buffer: header | descriptors | tile prefix
    uint8_t *d_buf = nullptr;
    size_t cap = 0;  // requests the buffer holds
    uint8_t *h_stage = nullptr;  // pinned staging of the same layout
    hipEvent_t staged = nullptr; // the last upload from h_stage has been consumed
    hipEvent_t done = nullptr;   // recorded after every (tracked) launch
    hipStream_t last_stream = nullptr;  // stream of the last tracked launch
    bool last_set = false;
    unsigned long long *d_counter = nullptr;  // [2] tile counters, one per direction
    int64_t ntiles_dir[2] = {0, 0};
    int64_t nslots_dir[2] = {0, 0};  // order-table slots per direction (ordered schedule)
    // tile order table (ordered schedule): device copy and pinned staging
    int32_t *d_order = nullptr;
    int32_t *h_order = nullptr;
    size_t order_cap = 0;
    bool staged_order = false;  // the uploaded table matches the current schedule
    int32_t lds_dir[2] = {0, 0};   // dynamic LDS per direction (the largest request's need)
    int32_t body_dir[2] = {0, 0};  // tile bodies each direction's requests take
    int32_t dirs = 0; // bit 0: has pack requests, bit 1: has unpack requests
    // captured launch
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;
    int graph_grid[2] = {-1, -1};
    int graph_policy = -1, graph_ordered = -1;
    int32_t graph_lds[2] = {-1, -1}, graph_body[2] = {-1, -1};
    uint8_t *graph_buf = nullptr;
    int32_t *graph_order = nullptr;
};

namespace mdt {
__global__ void batch_counter_reset(unsigned long long *counter) { *counter = 0ull; }
}  // namespace mdt

namespace {

constexpr size_t hdr_bytes() { return 256; }
constexpr size_t desc_off() { return hdr_bytes(); }
constexpr size_t tile_off(size_t cap) { return (desc_off() + cap * sizeof(ReqDesc) + 255) & ~(size_t)255; }
constexpr size_t buf_bytes(size_t cap) { return tile_off(cap) + (cap + 1) * sizeof(int64_t); }

void release_graph(mdt_batch_s *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->graph_grid[0] = b->graph_grid[1] = b->graph_policy = -1;
}

int ensure_capacity(mdt_batch_s *b, size_t n)
{
    if (n <= b->cap && b->d_buf) return MDT_SUCCESS;
    size_t cap = std::max<size_t>(64, b->cap);
    while (cap < n) cap *= 2;
    if (b->staged) (void)hipEventSynchronize(b->staged);
    (void)hipDeviceSynchronize();  // the old buffer may still be read by a launch in flight
    release_graph(b);
    if (b->d_buf) (void)hipFree(b->d_buf);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    b->d_buf = nullptr;
    b->h_stage = nullptr;
    b->cap = 0;
    hipError_t e = hipMalloc((void **)&b->d_buf, buf_bytes(cap));
    if (e != hipSuccess) {
        set_hip_error((int)e);
        return MDT_ERR_NO_MEM;
    }
    e = hipHostMalloc((void **)&b->h_stage, buf_bytes(cap), hipHostMallocDefault);
    if (e != hipSuccess) {
        set_hip_error((int)e);
        return MDT_ERR_NO_MEM;
    }
    b->cap = cap;
    return MDT_SUCCESS;
}

int init_device(mdt_batch_s *b)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_hip_error((int)e);
        return MDT_ERR_HIP;
    }
    if (b->device == dev) return MDT_SUCCESS;
    if (b->device >= 0) return MDT_ERR_STATE;  // a batch stays on the device it was first used on
    b->device = dev;
    if (hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || b->ncu <= 0)
        b->ncu = 256;
    if (hipMalloc((void **)&b->d_counter, 2 * sizeof(unsigned long long)) != hipSuccess) return MDT_ERR_NO_MEM;
    if (hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) return MDT_ERR_HIP;
    if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) return MDT_ERR_HIP;
    if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) return MDT_ERR_HIP;
    return MDT_SUCCESS;
}

// XCDs of the device: workgroup b of a launch runs on XCD b mod XCDS
// (round-robin dispatch), and each XCD has its own L2.
constexpr int XCDS = 8;
constexpr int64_t XCD_GROUP = 8;

// Typed-address order of each direction's tiles (the address a tile's first
// packed byte comes from or goes to).  With the static policy slot t of a
// direction runs on XCD t mod XCDS, so the sorted tiles are dealt out to the
// XCDs in groups of XCD_GROUP neighbours: tiles that touch the same lines
// share an L2, and every XCD still gets a spread of the whole address range
// (contiguous slices left whole faces on one XCD).
int build_order(mdt_batch_s *b, const ReqDesc *D, const int64_t *tile0, const BatchHeader &H)
{
    const int64_t T = b->cfg.tile_chunks;
    const int64_t total = H.ntiles_dir[0] + H.ntiles_dir[1];
    if (total > INT32_MAX / 2) return MDT_ERR_COUNT;
    // slots: tiles rounded up to a multiple of XCDS * XCD_GROUP per direction
    const size_t need = (size_t)(total + 2 * XCDS * XCD_GROUP);
    if (need > b->order_cap) {
        size_t cap = std::max<size_t>(need, 2 * b->order_cap);
        (void)hipDeviceSynchronize();  // a launch in flight may read the old table
        release_graph(b);
        if (b->d_order) (void)hipFree(b->d_order);
        if (b->h_order) (void)hipHostFree(b->h_order);
        b->d_order = nullptr;
        b->h_order = nullptr;
        b->order_cap = 0;
        hipError_t e = hipMalloc((void **)&b->d_order, cap * sizeof(int32_t));
        if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_order, cap * sizeof(int32_t), hipHostMallocDefault);
        if (e != hipSuccess) {
            set_hip_error((int)e);
            return MDT_ERR_NO_MEM;
        }
        b->order_cap = cap;
    }
    // requests in descriptor order are those of reqs filtered by direction
    std::vector<const BatchReq *> byk;
    for (int dir = 0; dir < 2; dir++)
        for (auto &r : b->reqs)
            if (r.d.unpack == dir) byk.push_back(&r);
    std::vector<std::pair<uint64_t, int32_t>> keys;
    int64_t slot0 = 0, k0 = 0;
    for (int dir = 0; dir < 2; dir++) {
        keys.clear();
        const int64_t nreq = H.nreq_dir[dir];
        for (int64_t k = k0; k < k0 + nreq; k++) {
            const ReqDesc &d = D[k];
            const DevLayout &L = byk[(size_t)k]->type->comp->host;
            for (int64_t t = tile0[k]; t < tile0[k + 1]; t++) {
                int64_t p = (t - tile0[k]) * d.tc * 16 - d.head;
                if (p < 0) p = 0;
                const uint64_t sp = (uint64_t)(d.off + p);
                Loc l;
                if (L.kind == KIND_CONTIG) l = locate<KIND_CONTIG>(L, sp, d.elem1);
                else if (L.kind == KIND_SINGLE) l = locate<KIND_SINGLE>(L, sp, d.elem1);
                else l = locate<KIND_MULTI>(L, sp, d.elem1);
                keys.emplace_back((uint64_t)((uintptr_t)d.typed + (uint64_t)l.addr), (int32_t)t);
            }
        }
        k0 += nreq;
        std::stable_sort(keys.begin(), keys.end(),
                         [](const std::pair<uint64_t, int32_t> &x, const std::pair<uint64_t, int32_t> &y) {
                             return x.first < y.first;
                         });
        const int64_t n = (int64_t)keys.size();
        int64_t nslots = n;
        if (b->cfg.policy != 1 && n > 0) {
            // groups g = 0, 1, ... of XCD_GROUP sorted tiles; group g runs on
            // XCD g mod XCDS.  Slot t (XCD t mod XCDS, i-th slot of that XCD)
            // takes position p of group (i / XCD_GROUP) * XCDS + XCD.
            const int64_t groups = (n + XCD_GROUP - 1) / XCD_GROUP;
            const int64_t rounds = (groups + XCDS - 1) / XCDS;
            nslots = rounds * XCDS * XCD_GROUP;
            for (int64_t t = 0; t < nslots; t++) {
                const int64_t x = t % XCDS, i = t / XCDS;
                const int64_t g = (i / XCD_GROUP) * XCDS + x;
                const int64_t p = g * XCD_GROUP + i % XCD_GROUP;
                b->h_order[slot0 + t] = p < n ? keys[(size_t)p].second : -1;
            }
        } else {
            for (int64_t t = 0; t < n; t++) b->h_order[slot0 + t] = keys[(size_t)t].second;
        }
        b->nslots_dir[dir] = nslots;
        slot0 += nslots;
    }
    return MDT_SUCCESS;
}

// Upload descriptors and the tile prefix (stream-ordered) if the batch changed.
int stage(mdt_batch_s *b, hipStream_t s)
{
    if (!b->dirty) return MDT_SUCCESS;
    int rc = ensure_capacity(b, b->reqs.size());
    if (rc) return rc;
    // the previous upload must have left the staging buffer
    hipError_t e = hipEventSynchronize(b->staged);
    if (e != hipSuccess) {
        set_hip_error((int)e);
        return MDT_ERR_HIP;
    }
    const int64_t T = b->cfg.tile_chunks;
    BatchHeader H{};
    H.tile_chunks = T;
    ReqDesc *D = (ReqDesc *)(b->h_stage + desc_off());
    int64_t *tile0 = (int64_t *)(b->h_stage + tile_off(b->cap));
    int64_t acc = 0;
    size_t k = 0;
    b->lds_dir[0] = b->lds_dir[1] = 0;
    b->body_dir[0] = b->body_dir[1] = 0;
    b->dirs = 0;
    // pack requests first, then unpack, each in the order they were added
    for (int dir = 0; dir < 2; dir++) {
        const int64_t acc0 = acc;
        int64_t min_run = INT64_MAX;
        for (size_t i = 0; i < b->reqs.size(); i++) {
            if (b->reqs[i].d.unpack != dir) continue;
            D[k] = b->reqs[i].d;
            D[k].tc = tile_chunks_of(b->cfg, b->reqs[i]);
            b->lds_dir[dir] = std::max(b->lds_dir[dir], b->reqs[i].lds);
            b->body_dir[dir] |= body_bits(D[k]);
            min_run = std::min(min_run, b->reqs[i].mean_run);
            tile0[k] = acc;
            acc += (D[k].nchunks + D[k].tc - 1) / D[k].tc;
            H.nreq_dir[dir]++;
            k++;
        }
        H.ntiles_dir[dir] = acc - acc0;
        b->ntiles_dir[dir] = acc - acc0;
        b->body_dir[dir] = dir_body(b->body_dir[dir], dir, min_run);
        if (acc > acc0) b->dirs |= 1 << dir;
    }
    tile0[k] = acc;
    b->nslots_dir[0] = b->nslots_dir[1] = 0;
    if (b->cfg.order) {
        rc = build_order(b, D, tile0, H);
        if (rc) return rc;
    }
    H.ordered = b->cfg.order ? 1 : 0;
    {
        int64_t packed = 0;
        for (auto &r : b->reqs)
            if (!r.d.unpack && !r.type2) packed += r.d.nbytes;
        H.keep_packed = packed <= KEEP_PACKED_MAX ? 1 : 0;
    }
    H.nslots_dir[0] = b->nslots_dir[0];
    H.nslots_dir[1] = b->nslots_dir[1];
    std::memcpy(b->h_stage, &H, sizeof H);
    size_t n = tile_off(b->cap) + (b->reqs.size() + 1) * sizeof(int64_t);
    e = hipMemcpyAsync(b->d_buf, b->h_stage, n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && b->cfg.order && b->nslots_dir[0] + b->nslots_dir[1] > 0)
        e = hipMemcpyAsync(b->d_order, b->h_order, (size_t)(b->nslots_dir[0] + b->nslots_dir[1]) * sizeof(int32_t),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(b->staged, s);
    if (e != hipSuccess) {
        set_hip_error((int)e);
        return MDT_ERR_HIP;
    }
    b->dirty = false;
    return MDT_SUCCESS;
}

// Workgroups of one direction's launch: wgs_per_cu per compute unit
// (persistent), or one per tile when wgs_per_cu is 0.
int grid_of(const mdt_batch_s *b, int dir)
{
    const int64_t n = b->cfg.order ? b->nslots_dir[dir] : b->ntiles_dir[dir];
    int64_t g = b->cfg.wgs_per_cu > 0 ? std::min<int64_t>((int64_t)b->ncu * b->cfg.wgs_per_cu, n) : n;
    return (int)std::min<int64_t>(std::max<int64_t>(1, g), INT32_MAX);
}

template <int POLICY, int UNPACK>
void launch_dir(mdt_batch_s *b, hipStream_t s, dim3 grid, size_t lds, unsigned long long *ctr, int body)
{
    const BatchHeader *H = (const BatchHeader *)b->d_buf;
    const ReqDesc *R = (const ReqDesc *)(b->d_buf + desc_off());
    const int64_t *tile0 = (const int64_t *)(b->d_buf + tile_off(b->cap));
    launch_batch_dir<POLICY, UNPACK>(grid, lds, s, H, R, tile0, b->d_order, ctr, body);
}

// Policy 3: every request with its single-request kernel (one launch per
// request; in a graph, one node per request), pack direction first.  The
// first failure stops the enqueue and is returned (requests already enqueued
// still run).
int enqueue_single(mdt_batch_s *b, hipStream_t s)
{
    for (int dir = 0; dir < 2; dir++) {
        for (const BatchReq &r : b->reqs) {
            if (r.d.unpack != dir) continue;
            DeviceTables *D = nullptr;
            int rc = device_tables(r.type->comp.get(), &D);
            if (rc) return rc;
            if (r.d.body == BODY_RELAY) {
                DeviceTables *D2 = nullptr;
                rc = device_tables(r.type2->comp.get(), &D2);
                if (rc) return rc;
                rc = launch_xfer(D->lay, make_args(r.d.typed, r.d.packed, r.d.off, r.d.nbytes), false, s);
                if (!rc) rc = launch_xfer(D2->lay, make_args(r.d.typed2, r.d.packed, r.d.off, r.d.nbytes), true, s);
            } else if (r.type2) {
                DeviceTables *D2 = nullptr;
                rc = device_tables(r.type2->comp.get(), &D2);
                if (rc) return rc;
                CopyArgs A{};
                A.src = r.d.typed;
                A.dst = r.d.packed;
                A.off = r.d.off;
                A.nbytes = r.d.nbytes;
                A.nchunks = (r.d.nbytes + 15) / 16;
                A.src_elem1 = r.d.elem1;
                A.dst_elem1 = r.d.elem1_2;
                rc = launch_copy(D->lay, D2->lay, A, s);
            } else {
                rc = launch_xfer(D->lay, make_args(r.d.typed, r.d.packed, r.d.off, r.d.nbytes), dir == 1, s);
            }
            if (rc) return rc;
        }
    }
    return MDT_SUCCESS;
}

int enqueue_kernels(mdt_batch_s *b, hipStream_t s)
{
    if (b->cfg.policy == 3) return enqueue_single(b, s);
    // one kernel per direction: a mixed batch runs its pack tiles, then its
    // unpack tiles
    for (int dir = 0; dir < 2; dir++) {
        if (!(b->dirs & (1 << dir))) continue;
        const dim3 grid((unsigned)grid_of(b, dir));
        const size_t lds = (size_t)b->lds_dir[dir];
        const int body = b->body_dir[dir];
        unsigned long long *ctr = b->d_counter + dir;
        if (b->cfg.policy == 1) {
            hipLaunchKernelGGL(batch_counter_reset, dim3(1), dim3(1), 0, s, ctr);
            if (dir) launch_dir<1, 1>(b, s, grid, lds, ctr, body);
            else launch_dir<1, 0>(b, s, grid, lds, ctr, body);
        } else if (b->cfg.policy == 2 &&
                   (int64_t)grid.x == (b->cfg.order ? b->nslots_dir[dir] : b->ntiles_dir[dir])) {
            // one tile (or slot) per workgroup: the loop-free variant (the
            // looping one below covers a grid too small for that)
            if (dir) launch_dir<2, 1>(b, s, grid, lds, ctr, body);
            else launch_dir<2, 0>(b, s, grid, lds, ctr, body);
        } else {
            if (dir) launch_dir<0, 1>(b, s, grid, lds, ctr, body);
            else launch_dir<0, 0>(b, s, grid, lds, ctr, body);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_hip_error((int)e);
            return MDT_ERR_HIP;
        }
    }
    return MDT_SUCCESS;
}

// A batch owns one descriptor buffer, one order table and one pair of tile
// counters; a launch on another stream than the previous one first waits
// (on the device) for the previous launch, so a new upload or counter reset
// never lands under a kernel that still reads them.  The server's batches
// stay on one stream and skip the bookkeeping (track = false).
int launch(mdt_batch_s *b, hipStream_t s, bool track = true)
{
    int rc = init_device(b);
    if (rc) return rc;
    if (track && b->last_set && s != b->last_stream) {
        hipError_t e = hipStreamWaitEvent(s, b->done, 0);
        if (e != hipSuccess) {
            set_hip_error((int)e);
            return MDT_ERR_HIP;
        }
    }
    rc = stage(b, s);
    if (rc) return rc;
    if (b->ntiles_dir[0] + b->ntiles_dir[1] == 0) return MDT_SUCCESS;
    const int g0 = (b->dirs & 1) ? grid_of(b, 0) : 0, g1 = (b->dirs & 2) ? grid_of(b, 1) : 0;
    if (!b->cfg.use_graph) {
        rc = enqueue_kernels(b, s);
    } else {
        if (!b->exec || b->graph_grid[0] != g0 || b->graph_grid[1] != g1 || b->graph_policy != b->cfg.policy ||
            b->graph_buf != b->d_buf || b->graph_lds[0] != b->lds_dir[0] || b->graph_lds[1] != b->lds_dir[1] ||
            b->graph_body[0] != b->body_dir[0] || b->graph_body[1] != b->body_dir[1] ||
            b->graph_ordered != b->cfg.order || b->graph_order != b->d_order ||
            (b->cfg.policy == 3 && b->graph_gen != b->gen)) {
            release_graph(b);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                rc = enqueue_kernels(b, b->cap_stream);
                e = hipStreamEndCapture(b->cap_stream, &g);  // ends the capture whatever rc is
            }
            if (e == hipSuccess && rc == MDT_SUCCESS) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (rc == MDT_SUCCESS && e != hipSuccess) {
                set_hip_error((int)e);
                rc = MDT_ERR_HIP;
            }
            if (rc) {
                b->exec = nullptr;
                return rc;
            }
            b->graph_grid[0] = g0;
            b->graph_grid[1] = g1;
            b->graph_policy = b->cfg.policy;
            b->graph_gen = b->gen;
            for (int d = 0; d < 2; d++) {
                b->graph_lds[d] = b->lds_dir[d];
                b->graph_body[d] = b->body_dir[d];
            }
            b->graph_buf = b->d_buf;
            b->graph_ordered = b->cfg.order;
            b->graph_order = b->d_order;
        }
        hipError_t e = hipGraphLaunch(b->exec, s);
        if (e != hipSuccess) {
            set_hip_error((int)e);
            rc = MDT_ERR_HIP;
        }
    }
    if (track) {
        // recorded even after a failed enqueue: what was enqueued still runs
        hipError_t e = hipEventRecord(b->done, s);
        if (e == hipSuccess) {
            b->last_stream = s;
            b->last_set = true;
        } else if (rc == MDT_SUCCESS) {
            set_hip_error((int)e);
            rc = MDT_ERR_HIP;
        }
    }
    return rc;
}

bool valid_batch(mdt_batch b) { return b && b->magic == BATCH_MAGIC; }

// ---- launches that allocate nothing ----------------------------------------
//
// mdt_batch_launch_noalloc runs a batch through a file-scope device array
// instead of the batch's own device buffers: the same layout (header,
// descriptors, tile prefix) for at most NOALLOC_MAX_REQ requests, plus the
// two tile counters.  Descriptors get there through staging kernels whose
// arguments carry them (STAGE_N per launch), so the call makes no host to
// device copy and no allocation.  Every call on a device shares that
// device's array.

constexpr int64_t NOALLOC_MAX_REQ = 1024;
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 10;
constexpr size_t NOALLOC_CTR_OFF = NOALLOC_SCRATCH_BYTES - 256;
constexpr int STAGE_N = 16;

struct StageChunk {
    int64_t first;        // index of the chunk's first descriptor
    int64_t n;            // descriptors in the chunk
    int64_t tile_end;     // the prefix entry after the chunk's last request (last chunk), else -1
    int64_t with_header;  // the chunk also writes the header
    BatchHeader H;
    ReqDesc d[STAGE_N];
    int64_t tile0[STAGE_N];
};

}  // namespace

static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

namespace mdt {
// one workgroup copies a chunk of descriptors (and the header) into place
__global__ __launch_bounds__(256) void noalloc_stage_kernel(uint8_t *buf, StageChunk c)
{
    const int t = threadIdx.x;
    uint64_t *R = (uint64_t *)(buf + desc_off());
    int64_t *tile0 = (int64_t *)(buf + tile_off((size_t)NOALLOC_MAX_REQ));
    constexpr int W = (int)(sizeof(ReqDesc) / 8);
    for (int k = t; k < (int)c.n * W; k += 256) R[(size_t)c.first * W + k] = ((const uint64_t *)c.d)[k];
    for (int i = t; i < (int)c.n; i += 256) tile0[c.first + i] = c.tile0[i];
    if (t == 0 && c.tile_end >= 0) tile0[c.first + c.n] = c.tile_end;
    if (c.with_header)
        for (int w = t; w < (int)(sizeof(BatchHeader) / 8); w += 256)
            ((uint64_t *)buf)[w] = ((const uint64_t *)&c.H)[w];
}
}  // namespace mdt

namespace {

static_assert(sizeof(ReqDesc) % 8 == 0 && sizeof(BatchHeader) % 8 == 0, "staged as 8-byte words");
static_assert(sizeof(StageChunk) <= 2048, "a chunk travels as kernel arguments");

struct NoallocDevice {
    uint8_t *ptr = nullptr;  // this device's copy of `scratch`
    int ncu = 0;
    bool ready = false;
};
std::mutex g_noalloc_mu;
NoallocDevice g_noalloc[64];

// The device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array).
int noalloc_scratch(int dev, NoallocDevice **out)
{
    if (dev < 0 || dev >= 64) return MDT_ERR_ARG;
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    NoallocDevice &d = g_noalloc[dev];
    if (!d.ready) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_hip_error((int)e);
            return MDT_ERR_HIP;
        }
        if (hipDeviceGetAttribute(&d.ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || d.ncu <= 0)
            d.ncu = 256;
        d.ptr = static_cast<uint8_t *>(p);
        d.ready = true;
    }
    *out = &d;
    return MDT_SUCCESS;
}

int launch_noalloc(mdt_batch_s *b, hipStream_t s)
{
    static_assert(NOALLOC_CTR_OFF >= buf_bytes(NOALLOC_MAX_REQ), "counters after the descriptor area");
    if ((int64_t)b->reqs.size() > NOALLOC_MAX_REQ) return MDT_ERR_NO_MEM;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_hip_error((int)e);
        return MDT_ERR_HIP;
    }
    NoallocDevice *nd = nullptr;
    int rc = noalloc_scratch(dev, &nd);
    if (rc) return rc;
    // every request's layout tables must already be on this device (they
    // are uploaded when a request is added): nothing is uploaded here
    for (const BatchReq &r : b->reqs) {
        DeviceTables *D = nullptr;
        rc = device_tables_resident(r.type->comp.get(), &D);
        if (rc) return rc;
        if ((uint64_t)(uintptr_t)D->d_lay != r.d.lay) return MDT_ERR_STATE;
        if (r.type2) {
            rc = device_tables_resident(r.type2->comp.get(), &D);
            if (rc) return rc;
        }
    }
    if (b->cfg.policy == 3) return enqueue_single(b, s);  // per-request kernels use no scratch
    const int64_t T = b->cfg.tile_chunks;
    BatchHeader H{};
    H.tile_chunks = T;
    int32_t lds_dir[2] = {0, 0}, body_dir[2] = {0, 0};
    int64_t min_run[2] = {INT64_MAX, INT64_MAX};
    int64_t packed = 0;
    for (const BatchReq &r : b->reqs) {
        const int dir = r.d.unpack;
        H.nreq_dir[dir]++;
        H.ntiles_dir[dir] += (r.d.nchunks + T - 1) / T;  // request order: every request at T
        lds_dir[dir] = std::max(lds_dir[dir], r.lds);
        body_dir[dir] |= body_bits(r.d);
        min_run[dir] = std::min(min_run[dir], r.mean_run);
        if (!dir && !r.type2) packed += r.d.nbytes;
    }
    for (int dir = 0; dir < 2; dir++) body_dir[dir] = dir_body(body_dir[dir], dir, min_run[dir]);
    H.keep_packed = packed <= KEEP_PACKED_MAX ? 1 : 0;
    if (H.ntiles_dir[0] + H.ntiles_dir[1] > INT32_MAX) return MDT_ERR_COUNT;
    // stage the descriptors, pack requests first, in chunks
    StageChunk c{};
    c.H = H;
    c.with_header = 1;
    int64_t k = 0, acc = 0;
    const int64_t nreq = (int64_t)b->reqs.size();
    auto flush = [&](bool last) {
        c.tile_end = last ? acc : -1;
        hipLaunchKernelGGL(noalloc_stage_kernel, dim3(1), dim3(256), 0, s, nd->ptr, c);
        c.first += c.n;
        c.n = 0;
        c.with_header = 0;
    };
    for (int dir = 0; dir < 2; dir++)
        for (const BatchReq &r : b->reqs) {
            if (r.d.unpack != dir) continue;
            c.d[c.n] = r.d;
            c.d[c.n].tc = T;
            c.tile0[c.n] = acc;
            acc += (r.d.nchunks + T - 1) / T;
            c.n++;
            k++;
            if (c.n == STAGE_N || k == nreq) flush(k == nreq);
        }
    if (nreq == 0) flush(true);
    const BatchHeader *Hd = (const BatchHeader *)nd->ptr;
    const ReqDesc *R = (const ReqDesc *)(nd->ptr + desc_off());
    const int64_t *tile0 = (const int64_t *)(nd->ptr + tile_off((size_t)NOALLOC_MAX_REQ));
    unsigned long long *ctr = (unsigned long long *)(nd->ptr + NOALLOC_CTR_OFF);
    for (int dir = 0; dir < 2; dir++) {
        const int64_t nt = H.ntiles_dir[dir];
        if (nt == 0) continue;
        int64_t g = b->cfg.wgs_per_cu > 0 ? std::min<int64_t>((int64_t)nd->ncu * b->cfg.wgs_per_cu, nt) : nt;
        const dim3 grid((unsigned)std::max<int64_t>(1, g));
        const size_t lds = (size_t)lds_dir[dir];
        if (b->cfg.policy == 1) {
            // the dynamic split's counter starts at zero (a kernel, not a memset)
            hipLaunchKernelGGL(batch_counter_reset, dim3(1), dim3(1), 0, s, ctr + dir);
            if (dir) launch_batch_dir<1, 1>(grid, lds, s, Hd, R, tile0, nullptr, ctr + dir, body_dir[dir]);
            else launch_batch_dir<1, 0>(grid, lds, s, Hd, R, tile0, nullptr, ctr + dir, body_dir[dir]);
        } else if (b->cfg.policy == 2 && (int64_t)grid.x == nt) {
            if (dir) launch_batch_dir<2, 1>(grid, lds, s, Hd, R, tile0, nullptr, ctr + dir, body_dir[dir]);
            else launch_batch_dir<2, 0>(grid, lds, s, Hd, R, tile0, nullptr, ctr + dir, body_dir[dir]);
        } else {
            if (dir) launch_batch_dir<0, 1>(grid, lds, s, Hd, R, tile0, nullptr, ctr + dir, body_dir[dir]);
            else launch_batch_dir<0, 0>(grid, lds, s, Hd, R, tile0, nullptr, ctr + dir, body_dir[dir]);
        }
    }
    e = hipGetLastError();
    if (e != hipSuccess) {
        set_hip_error((int)e);
        return MDT_ERR_HIP;
    }
    return MDT_SUCCESS;
}

bool valid_cfg(const mdt_batch_config &c)
{
    bool tc = c.tile_chunks == 256 || c.tile_chunks == 512 || c.tile_chunks == 1024 || c.tile_chunks == 2048 ||
              c.tile_chunks == 4096;
    return tc && c.wgs_per_cu >= 0 && c.wgs_per_cu <= 16 && c.policy >= 0 && c.policy <= 3 &&
           (c.policy < 2 || c.wgs_per_cu == 0) && (c.policy != 3 || c.order == 0) &&
           (c.use_graph == 0 || c.use_graph == 1) && (c.order == 0 || c.order == 1);
}

// The tile body a request takes (the same choice as the single-request
// launch) and the dynamic LDS it needs.
int body_of(const DevLayout &L, const XferArgs &A, bool unpack, int32_t *lds)
{
    if (use_dense(L, A, unpack)) {
        *lds = L.rec.lds_bytes;
        return BODY_DENSE;
    }
    if (use_runs(L)) {
        *lds = (int32_t)sizeof(RunsCache);
        return BODY_RUNS;
    }
    *lds = 0;
    return BODY_CHUNK;
}

int add_req(mdt_batch b, TypeNode *t, const ReqDesc &d, int32_t lds, TypeNode *t2 = nullptr)
{
    try {
        retain(t);
        if (t2) retain(t2);
        const int64_t runs = t->comp ? t->comp->nruns : 0;
        b->reqs.push_back({t, d, lds, t2, runs > 0 ? t->size / runs : INT64_MAX});
    } catch (...) {
        release(t);
        if (t2) release(t2);
        return MDT_ERR_NO_MEM;
    }
    b->dirty = true;
    b->gen++;
    return MDT_SUCCESS;
}

}  // namespace

namespace {

// ---- the autotuner and its cache ----------------------------------------
//
// Candidates: tile size x workgroups per CU x split policy x tile order x
// graph replay (the grid below).  Each candidate runs the set of batches in
// turn -- a caller's rotating copies, so the timing sees the inputs as they
// run, out of cache -- once to warm up (uploads, graph capture) and then
// TUNE_REPS times; the median set time decides.  With MDT_AUTOTUNE_CACHE
// naming a file, a choice is kept there under the batch's shape and reused
// (no timing) by later tunings of the same shape on the same kind of device.

constexpr int TUNE_REPS = 5;

uint64_t fnv1a(uint64_t h, uint64_t v)
{
    for (int i = 0; i < 8; i++) {
        h ^= (v >> (8 * i)) & 0xff;
        h *= 1099511628211ull;
    }
    return h;
}

// The shape of a batch: per request its direction, body, layout kind, type
// size, runs per element and packed bytes (to a power of two), in request
// order; plus the device's compute units and the library version.
std::string shape_key(mdt_batch_s *b, int ncu)
{
    uint64_t h = 1469598103934665603ull;
    h = fnv1a(h, (uint64_t)mdt_version());
    h = fnv1a(h, (uint64_t)ncu);
    for (const BatchReq &r : b->reqs) {
        h = fnv1a(h, ((uint64_t)r.d.unpack << 48) | ((uint64_t)r.d.body << 32) | (uint64_t)(uint32_t)r.d.kind);
        h = fnv1a(h, (uint64_t)r.type->size);
        h = fnv1a(h, (uint64_t)(r.type->comp ? r.type->comp->nruns : 0));
        h = fnv1a(h, (uint64_t)(64 - __builtin_clzll((uint64_t)r.d.nbytes | 1)));
        if (r.type2) h = fnv1a(h, (uint64_t)r.type2->size);
    }
    char buf[40];
    std::snprintf(buf, sizeof buf, "%016llx-%zu", (unsigned long long)h, b->reqs.size());
    return buf;
}

// Cache file: one entry per line, `"key": [tile_chunks, wgs_per_cu, policy,
// use_graph, order]`, inside one JSON object.
std::mutex g_cache_mu;

bool cache_lookup(const char *path, const std::string &key, mdt_batch_config *c)
{
    std::lock_guard<std::mutex> g(g_cache_mu);
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    const std::string want = "\"" + key + "\"";
    while (!found && std::fgets(line, sizeof line, f)) {
        const char *p = std::strstr(line, want.c_str());
        if (!p) continue;
        mdt_batch_config x{};
        if (std::sscanf(p + want.size(), " : [%d, %d, %d, %d, %d]", &x.tile_chunks, &x.wgs_per_cu, &x.policy,
                        &x.use_graph, &x.order) == 5 &&
            valid_cfg(x)) {
            *c = x;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, const mdt_batch_config &c)
{
    std::lock_guard<std::mutex> g(g_cache_mu);
    std::vector<std::string> keep;
    if (FILE *f = std::fopen(path, "r")) {
        char line[256];
        const std::string own = "\"" + key + "\"";
        while (std::fgets(line, sizeof line, f)) {
            std::string l(line);
            if (l.find("\": [") == std::string::npos || l.find(own) != std::string::npos) continue;
            while (!l.empty() && (l.back() == '\n' || l.back() == ',' || l.back() == ' ')) l.pop_back();
            keep.push_back(l);
        }
        std::fclose(f);
    }
    char buf[160];
    std::snprintf(buf, sizeof buf, "  \"%s\": [%d, %d, %d, %d, %d]", key.c_str(), c.tile_chunks, c.wgs_per_cu,
                  c.policy, c.use_graph, c.order);
    keep.push_back(buf);
    // a temporary of this process's own, replacing the file in one step: two
    // processes storing at once each leave a whole file (the later one wins)
    const std::string tmp = std::string(path) + ".tmp." + std::to_string((long long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fputs("{\n", f);
    for (size_t i = 0; i < keep.size(); i++) std::fprintf(f, "%s%s\n", keep[i].c_str(), i + 1 < keep.size() ? "," : "");
    std::fputs("}\n", f);
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

int autotune_set(int n, mdt_batch *bs, hipStream_t s, mdt_batch_config *best)
{
    int rc = init_device(bs[0]);
    if (rc) return rc;
    const char *path = std::getenv("MDT_AUTOTUNE_CACHE");
    std::string key;
    if (path && *path) {
        key = shape_key(bs[0], bs[0]->ncu);
        mdt_batch_config c{};
        if (cache_lookup(path, key, &c)) {
            for (int i = 0; i < n; i++) mdt_batch_set_config(bs[i], &c);
            if (best) *best = c;
            return MDT_SUCCESS;
        }
    }
    std::vector<mdt_batch_config> keep((size_t)n);
    for (int i = 0; i < n; i++) keep[(size_t)i] = bs[i]->cfg;
    mdt_batch_config win = keep[0];
    float win_ms = 1e30f;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MDT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MDT_ERR_HIP;
    }
    const int tiles[] = {256, 1024, 4096};
    const int occ[] = {0, 2, 4, 8};  // 0: one workgroup per tile
    auto run_set = [&]() {
        for (int i = 0; i < n; i++) {
            int r = launch(bs[i], s);
            if (r) return r;
        }
        return (int)MDT_SUCCESS;
    };
    for (int graph = 0; graph < 2 && !rc; graph++)
        for (int ord = 0; ord < 2 && !rc; ord++)
            for (int policy = 0; policy < 4 && !rc; policy++)
                for (int tc : tiles)
                    for (int w : occ) {
                        if (rc) break;
                        if (policy == 1 && w == 0) continue;  // nothing to balance with a workgroup per tile
                        if (policy == 2 && w != 0) continue;  // the loop-free kernel takes one tile per workgroup
                        // single-request kernels: their own tiles, no order
                        if (policy == 3 && (w != 0 || tc != 1024 || ord != 0)) continue;
                        mdt_batch_config c{tc, w, policy, graph, ord};
                        for (int i = 0; i < n; i++) mdt_batch_set_config(bs[i], &c);
                        rc = run_set();  // warm-up (uploads, graph capture)
                        if (rc) break;
                        float ms[TUNE_REPS];
                        for (int k = 0; k < TUNE_REPS && !rc; k++) {
                            (void)hipEventRecord(e0, s);
                            rc = run_set();
                            (void)hipEventRecord(e1, s);
                            (void)hipEventSynchronize(e1);
                            (void)hipEventElapsedTime(&ms[k], e0, e1);
                        }
                        if (rc) break;
                        std::sort(ms, ms + TUNE_REPS);
                        if (ms[TUNE_REPS / 2] < win_ms) {
                            win_ms = ms[TUNE_REPS / 2];
                            win = c;
                        }
                    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        for (int i = 0; i < n; i++) mdt_batch_set_config(bs[i], &keep[(size_t)i]);
        return rc;
    }
    for (int i = 0; i < n; i++) mdt_batch_set_config(bs[i], &win);
    if (path && *path) cache_store(path, key, win);
    if (best) *best = win;
    return MDT_SUCCESS;
}

}  // namespace

namespace mdt {
// used by the serving loop
int batch_launch_internal(mdt_batch b, hipStream_t s) { return launch(b, s, false); }
}  // namespace mdt

extern "C" {

MDT_API int mdt_batch_create(mdt_batch *out)
{
    if (!out) return MDT_ERR_ARG;
    auto *b = new (std::nothrow) mdt_batch_s();
    if (!b) return MDT_ERR_NO_MEM;
    *out = b;
    return MDT_SUCCESS;
}

MDT_API int mdt_batch_clear(mdt_batch b)
{
    if (!valid_batch(b)) return MDT_ERR_ARG;
    for (auto &r : b->reqs) {
        release(r.type);
        if (r.type2) release(r.type2);
    }
    b->reqs.clear();
    b->dirty = true;
    b->gen++;
    return MDT_SUCCESS;
}

MDT_API int mdt_batch_free(mdt_batch *pb)
{
    if (!pb || !valid_batch(*pb)) return MDT_ERR_ARG;
    mdt_batch b = *pb;
    if (b->device >= 0) (void)hipDeviceSynchronize();  // launches in flight read the buffers
    mdt_batch_clear(b);
    release_graph(b);
    if (b->d_buf) (void)hipFree(b->d_buf);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    if (b->d_counter) (void)hipFree(b->d_counter);
    if (b->d_order) (void)hipFree(b->d_order);
    if (b->h_order) (void)hipHostFree(b->h_order);
    if (b->staged) (void)hipEventDestroy(b->staged);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    b->magic = 0;
    delete b;
    *pb = nullptr;
    return MDT_SUCCESS;
}

MDT_API int mdt_batch_add_pack(mdt_batch b, const void *inbuf, mdt_count incount, mdt_type t, mdt_count inoffset,
                               void *outbuf, mdt_count max_pack_bytes, mdt_count *actual_pack_bytes)
{
    if (!valid_batch(b) || !actual_pack_bytes || inoffset < 0 || max_pack_bytes < -1) return MDT_ERR_ARG;
    Compiled *C;
    DeviceTables *D;
    int64_t total;
    int rc = prepare(t, incount, &C, &D, &total);
    if (rc) return rc;
    int64_t n = std::max<int64_t>(0, total - inoffset);
    if (max_pack_bytes >= 0) n = std::min<int64_t>(n, max_pack_bytes);
    if (n > 0 && (!inbuf || !outbuf)) return MDT_ERR_ARG;
    if (n > 0) {
        XferArgs A = make_args(inbuf, outbuf, inoffset, n);
        A.elem1 = A.off + A.nbytes <= D->lay.size;
        int32_t lds = 0;
        const int body = body_of(D->lay, A, false, &lds);
        ReqDesc d{(uint64_t)(uintptr_t)D->d_lay, A.typed, A.packed, A.off, A.nbytes, A.head, A.nchunks, 0, D->lay.kind, A.elem1, body};
        rc = add_req(b, reinterpret_cast<TypeNode *>(t), d, lds);
        if (rc) return rc;
    }
    *actual_pack_bytes = n;
    return MDT_SUCCESS;
}

MDT_API int mdt_batch_add_unpack(mdt_batch b, const void *inbuf, mdt_count insize, void *outbuf,
                                 mdt_count outcount, mdt_type t, mdt_count outoffset, mdt_count *actual_unpack_bytes)
{
    if (!valid_batch(b) || !actual_unpack_bytes || insize < 0 || outoffset < 0) return MDT_ERR_ARG;
    Compiled *C;
    DeviceTables *D;
    int64_t total;
    int rc = prepare(t, outcount, &C, &D, &total);
    if (rc) return rc;
    if (insize > std::max<int64_t>(0, total - outoffset)) return MDT_ERR_TRUNCATE;
    rc = check_unpack_overlap(C, outcount);
    if (rc) return rc;
    if (insize > 0 && (!inbuf || !outbuf)) return MDT_ERR_ARG;
    if (insize > 0) {
        XferArgs A = make_args(outbuf, const_cast<void *>(inbuf), outoffset, insize);
        A.elem1 = A.off + A.nbytes <= D->lay.size;
        int32_t lds = 0;
        const int body = body_of(D->lay, A, true, &lds);
        ReqDesc d{(uint64_t)(uintptr_t)D->d_lay, A.typed, A.packed, A.off, A.nbytes, A.head, A.nchunks, 1, D->lay.kind, A.elem1, body};
        rc = add_req(b, reinterpret_cast<TypeNode *>(t), d, lds);
        if (rc) return rc;
    }
    *actual_unpack_bytes = insize;
    return MDT_SUCCESS;
}

MDT_API int mdt_batch_add_copy(mdt_batch b, const void *src, mdt_count srccount, mdt_type srctype, void *dst,
                               mdt_count dstcount, mdt_type dsttype, mdt_count offset, mdt_count max_bytes,
                               mdt_count *actual)
{
    if (!valid_batch(b) || !actual || offset < 0 || max_bytes < -1) return MDT_ERR_ARG;
    Compiled *Cs, *Cd;
    DeviceTables *Ds = nullptr, *Dd = nullptr;
    int64_t total_s, total_d;
    int rc = prepare(srctype, srccount, &Cs, nullptr, &total_s);
    if (rc) return rc;
    rc = prepare(dsttype, dstcount, &Cd, nullptr, &total_d);
    if (rc) return rc;
    int64_t n = std::max<int64_t>(0, total_s - offset);
    if (max_bytes >= 0) n = std::min<int64_t>(n, max_bytes);
    if (n > std::max<int64_t>(0, total_d - offset)) return MDT_ERR_TRUNCATE;
    rc = check_unpack_overlap(Cd, dstcount);
    if (rc) return rc;
    if (n > 0 && (!src || !dst)) return MDT_ERR_ARG;
    if (n > 0) {
        rc = device_tables(Cs, &Ds);
        if (rc) return rc;
        rc = device_tables(Cd, &Dd);
        if (rc) return rc;
        ReqDesc d{};
        d.lay = (uint64_t)(uintptr_t)Ds->d_lay;
        d.typed = (const uint8_t *)src;
        d.packed = (uint8_t *)dst;
        d.off = offset;
        d.nbytes = n;
        d.head = 0;
        d.nchunks = (n + 15) / 16;
        d.unpack = 0;
        d.kind = Ds->lay.kind;
        d.elem1 = offset + n <= Ds->lay.size;
        d.body = BODY_COPY;
        d.lay2 = (uint64_t)(uintptr_t)Dd->d_lay;
        d.kind2 = Dd->lay.kind;
        d.elem1_2 = offset + n <= Dd->lay.size;
        rc = add_req(b, reinterpret_cast<TypeNode *>(srctype), d, 0, reinterpret_cast<TypeNode *>(dsttype));
        if (rc) return rc;
    }
    *actual = n;
    return MDT_SUCCESS;
}

MDT_API int mdt_batch_add_relay(mdt_batch b, const void *src, mdt_count srccount, mdt_type srctype, void *packed,
                                void *dst, mdt_count dstcount, mdt_type dsttype, mdt_count offset, mdt_count max_bytes,
                                mdt_count *actual)
{
    if (!valid_batch(b) || !actual || offset < 0 || max_bytes < -1) return MDT_ERR_ARG;
    Compiled *Cs, *Cd;
    DeviceTables *Ds = nullptr, *Dd = nullptr;
    int64_t total_s, total_d;
    int rc = prepare(srctype, srccount, &Cs, &Ds, &total_s);
    if (rc) return rc;
    rc = prepare(dsttype, dstcount, &Cd, &Dd, &total_d);
    if (rc) return rc;
    int64_t n = std::max<int64_t>(0, total_s - offset);
    if (max_bytes >= 0) n = std::min<int64_t>(n, max_bytes);
    if (n > std::max<int64_t>(0, total_d - offset)) return MDT_ERR_TRUNCATE;
    rc = check_unpack_overlap(Cd, dstcount);
    if (rc) return rc;
    if (n > 0 && (!src || !packed || !dst)) return MDT_ERR_ARG;
    if (n > 0) {
        XferArgs A = make_args(src, packed, offset, n);
        A.elem1 = A.off + A.nbytes <= Ds->lay.size;
        XferArgs U = make_args(dst, packed, offset, n);
        U.elem1 = U.off + U.nbytes <= Dd->lay.size;
        int32_t lds_p = 0, lds_u = 0;
        ReqDesc d{};
        d.lay = (uint64_t)(uintptr_t)Ds->d_lay;
        d.typed = A.typed;
        d.packed = A.packed;
        d.off = A.off;
        d.nbytes = A.nbytes;
        d.head = A.head;
        d.nchunks = A.nchunks;
        d.unpack = 0;
        d.kind = Ds->lay.kind;
        d.elem1 = A.elem1;
        d.body = BODY_RELAY;
        d.lay2 = (uint64_t)(uintptr_t)Dd->d_lay;
        d.kind2 = Dd->lay.kind;
        d.elem1_2 = U.elem1;
        d.typed2 = U.typed;
        d.pbody = body_of(Ds->lay, A, false, &lds_p);
        // the unpack side reads back only its own tile's packed chunks: the
        // record view's unpack stages packed bytes of neighbouring records,
        // which other workgroups may not have packed yet, so it is not used
        d.ubody = body_of(Dd->lay, U, true, &lds_u);
        if (d.ubody == BODY_DENSE) {
            d.ubody = use_runs(Dd->lay) ? BODY_RUNS : BODY_CHUNK;
            lds_u = d.ubody == BODY_RUNS ? (int32_t)sizeof(RunsCache) : 0;
        }
        rc = add_req(b, reinterpret_cast<TypeNode *>(srctype), d, std::max(lds_p, lds_u),
                     reinterpret_cast<TypeNode *>(dsttype));
        if (rc) return rc;
    }
    *actual = n;
    return MDT_SUCCESS;
}

MDT_API int mdt_batch_set_config(mdt_batch b, const mdt_batch_config *cfg)
{
    if (!valid_batch(b) || !cfg || !valid_cfg(*cfg)) return MDT_ERR_ARG;
    // the tile prefix depends on the tile size, the order table on the order
    // and (through the XCD slicing) the policy
    if (cfg->tile_chunks != b->cfg.tile_chunks || cfg->order != b->cfg.order ||
        (cfg->order && cfg->policy != b->cfg.policy))
        b->dirty = true;
    b->cfg = *cfg;
    return MDT_SUCCESS;
}

MDT_API int mdt_batch_get_config(mdt_batch b, mdt_batch_config *cfg)
{
    if (!valid_batch(b) || !cfg) return MDT_ERR_ARG;
    *cfg = b->cfg;
    return MDT_SUCCESS;
}

MDT_API int mdt_batch_launch(mdt_batch b, mdt_stream s, mdt_request *req)
{
    mdt::TraceRange trace_("mdt_batch_launch");
    if (!valid_batch(b) || !s || s->magic != STREAM_MAGIC) return MDT_ERR_ARG;
    int rc = launch(b, s->s);
    if (rc) return rc;
    return request_from_stream(s->s, req, s);
}

MDT_API int mdt_batch_launch_noalloc(mdt_batch b, mdt_stream s)
{
    mdt::TraceRange trace_("mdt_batch_launch_noalloc");
    if (!valid_batch(b) || !s || s->magic != STREAM_MAGIC) return MDT_ERR_ARG;
    return launch_noalloc(b, s->s);
}

MDT_API int mdt_batch_autotune_set(int n, mdt_batch *batches, mdt_stream s, mdt_batch_config *best)
{
    mdt::TraceRange trace_("mdt_batch_autotune_set");
    if (n <= 0 || !batches || !s || s->magic != STREAM_MAGIC) return MDT_ERR_ARG;
    for (int i = 0; i < n; i++)
        if (!valid_batch(batches[i])) return MDT_ERR_ARG;
    return autotune_set(n, batches, s->s, best);
}

MDT_API int mdt_batch_autotune(mdt_batch b, mdt_stream s, mdt_batch_config *best)
{
    mdt::TraceRange trace_("mdt_batch_autotune");
    if (!valid_batch(b) || !s || s->magic != STREAM_MAGIC) return MDT_ERR_ARG;
    return autotune_set(1, &b, s->s, best);
}

}  // extern "C"
