// batch_kernel.h -- the batch kernel: descriptors, tile bodies, and the
// launch of one direction.  Its variants are compiled in six translation
// units (launch policy x direction, batch_variants.hip) so they build
// in parallel; batch.hip holds the host side.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"
#include "xfer.h"

namespace mdt {

struct ReqDesc {
    uint64_t lay;          // address of the device copy of the request's layout program
    const uint8_t *typed;  // typed origin (copy: the source origin)
    uint8_t *packed;       // packed buffer (copy: the destination origin)
    int64_t off, nbytes, head, nchunks;
    int32_t unpack, kind;
    int32_t elem1, body;  // BODY_DENSE, BODY_RUNS, BODY_CHUNK or BODY_COPY
    uint64_t lay2;         // copy, relay: the destination's layout program
    int32_t kind2, elem1_2;
    int64_t tc;            // 16-byte chunks per tile of this request
    const uint8_t *typed2; // relay: the destination origin
    int32_t pbody, ubody;  // relay: tile bodies of its pack and its unpack
};

// Tile bodies a batch kernel carries (a bit set): a kernel compiled for one
// body needs only that body's registers, so a direction whose requests all
// take one path runs at that path's occupancy.
constexpr int BODY_DENSE = 1;  // record view, LDS-staged
constexpr int BODY_RUNS = 2;   // run tables, LDS-cached group slice
constexpr int BODY_CHUNK = 4;  // chunk path
constexpr int BODY_ALL = 7;
constexpr int BODY_COPY = 8;   // typed copy (runs with the pack direction)
constexpr int BODY_RELAY = 16; // pack, then unpack of the same packed bytes (runs with the pack direction)
constexpr int BODY_CACHED = 32; // with BODY_CHUNK alone, pack: gathers load through the caches

// Descriptors are stored pack requests first, so each direction's tiles
// form one range: [0, ntiles_dir[0]) for pack, then unpack.
struct BatchHeader {
    int64_t nreq_dir[2];    // requests per direction
    int64_t ntiles_dir[2];  // tiles per direction
    int64_t tile_chunks;
    int64_t ordered;        // 1: slots map to tiles through the order table
    int64_t nslots_dir[2];  // order-table slots per direction (>= tiles; -1 entries are empty)
    int64_t keep_packed;    // the pack direction's output fits KEEP_PACKED_MAX: cached stores
};

// Chunks [c0, cend) of one request, with the single-request bodies.
template <int KS>
__device__ __forceinline__ void copy_tile_kd(const DevLayout &Ls, const DevLayout &Ld, int kd, const CopyArgs &A,
                                             int64_t c0, int64_t cend)
{
    if (kd == KIND_CONTIG) copy_tile4<KS, KIND_CONTIG>(Ls, Ld, A, c0, cend);
    else if (kd == KIND_SINGLE) copy_tile4<KS, KIND_SINGLE>(Ls, Ld, A, c0, cend);
    else copy_tile4<KS, KIND_MULTI>(Ls, Ld, A, c0, cend);
}

template <int UNPACK, int BODY>
__device__ __forceinline__ void run_tile(const DevLayout &L, const XferArgs &A, int body, int kind, int64_t c0,
                                         int64_t cend, uint8_t *lds_dyn, const ReqDesc &D)
{
    if ((BODY & BODY_RELAY) && body == BODY_RELAY) {
        // the tile's chunks are packed, then unpacked from the packed buffer
        // by the same workgroup: after the barrier every lane sees what the
        // others stored, still in the cache
        constexpr int SUB = BODY & BODY_ALL;
        XferArgs P = A;
        P.keep = 1;
        run_tile<0, SUB>(L, P, D.pbody, kind, c0, cend, lds_dyn, D);
        __syncthreads();
        const DevLayout &L2 = *(const DevLayout *)(const __attribute__((address_space(4))) DevLayout *)(uintptr_t)D.lay2;
        XferArgs U = A;
        U.typed = D.typed2;
        U.elem1 = D.elem1_2;
        run_tile<1, SUB>(L2, U, D.ubody, D.kind2, c0, cend, lds_dyn, D);
        return;
    }
    if ((BODY & BODY_COPY) && body == BODY_COPY) {
        const DevLayout &Ld = *(const DevLayout *)(const __attribute__((address_space(4))) DevLayout *)(uintptr_t)D.lay2;
        CopyArgs C;
        C.src = A.typed;
        C.dst = A.packed;
        C.off = A.off;
        C.nbytes = A.nbytes;
        C.nchunks = A.nchunks;
        C.src_elem1 = A.elem1;
        C.dst_elem1 = D.elem1_2;
        for (int64_t s0 = c0; s0 < cend; s0 += 1024) {
            int64_t s1 = s0 + 1024 < cend ? s0 + 1024 : cend;
            if (kind == KIND_CONTIG) copy_tile_kd<KIND_CONTIG>(L, Ld, D.kind2, C, s0, s1);
            else if (kind == KIND_SINGLE) copy_tile_kd<KIND_SINGLE>(L, Ld, D.kind2, C, s0, s1);
            else copy_tile_kd<KIND_MULTI>(L, Ld, D.kind2, C, s0, s1);
        }
        return;
    }
    if ((BODY & BODY_DENSE) && body == BODY_DENSE) {
        // sub-tiles sized to the type's LDS budget; LDS is reused between them
        const int64_t st = L.rec.tile_chunks;
        for (int64_t s0 = c0; s0 < cend; s0 += st) {
            int64_t s1 = s0 + st < cend ? s0 + st : cend;
            if (UNPACK) dense_unpack_tile(L, A, s0, s1, lds_dyn);
            else dense_pack_tile(L, A, s0, s1, lds_dyn);
            __syncthreads();
        }
        return;
    }
    if ((BODY & BODY_RUNS) && body == BODY_RUNS) {
        RunsCache &C = *reinterpret_cast<RunsCache *>(lds_dyn);
        for (int64_t s0 = c0; s0 < cend; s0 += 1024) {
            int64_t s1 = s0 + 1024 < cend ? s0 + 1024 : cend;
            runs_tile<UNPACK != 0>(L, A, s0, s1, C);
            __syncthreads();  // the cache is refilled for the next sub-tile
        }
        return;
    }
    if (BODY & BODY_CHUNK) {
        for (int64_t s0 = c0; s0 < cend; s0 += 1024) {
            int64_t s1 = s0 + 1024 < cend ? s0 + 1024 : cend;
            if (UNPACK) {
                if (kind == KIND_CONTIG) unpack_tile4<KIND_CONTIG>(L, A, s0, s1);
                else if (kind == KIND_SINGLE) unpack_tile4<KIND_SINGLE>(L, A, s0, s1);
                else unpack_tile4<KIND_MULTI>(L, A, s0, s1);
            } else {
                constexpr bool CACHED = (BODY & BODY_CACHED) != 0;
                if (kind == KIND_CONTIG) pack_tile4<KIND_CONTIG, CACHED>(L, A, s0, s1);
                else if (kind == KIND_SINGLE) pack_tile4<KIND_SINGLE, CACHED>(L, A, s0, s1);
                else pack_tile4<KIND_MULTI, CACHED>(L, A, s0, s1);
            }
        }
    }
}

// resets a dynamic split's tile counter before the launch (defined in batch.hip)
__global__ void batch_counter_reset(unsigned long long *counter);

// The same value in every lane, as a scalar (the tile index a workgroup
// works on is uniform; saying so keeps the request lookup and the layout
// reads on the scalar unit).
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A layout program read through the constant address space: it does not
// change while a kernel runs, so uniform reads of it become scalar loads, as
// they are for a layout passed by value as a kernel argument.
__device__ __forceinline__ const DevLayout &const_layout(uint64_t addr)
{
    return *(const DevLayout *)(const __attribute__((address_space(4))) DevLayout *)(uintptr_t)addr;
}

// Batch kernel for one direction.  POLICY 0: tile t = blockIdx.x + k *
// gridDim.x; POLICY 1: tiles taken from an atomic counter; POLICY 2: one
// tile (or order-table slot) per workgroup, with no loop, so no loop state
// holds scalar registers the tile bodies need.  Every workgroup leaves the
// loop once the tile index passes the direction's last tile.
template <int POLICY, int UNPACK, int BODY>
__global__ __launch_bounds__(256) void batch_kernel(const BatchHeader *__restrict__ H,
                                                    const ReqDesc *__restrict__ R,
                                                    const int64_t *__restrict__ tile0,
                                                    const int32_t *__restrict__ order,
                                                    unsigned long long *counter)
{
    extern __shared__ __align__(16) uint8_t lds_dyn[];
    __shared__ int64_t s_t;
    const bool ordered = H->ordered != 0;
    // this direction's requests [r0, r1) and index range [t_begin, t_end):
    // tiles, or slots of the order table
    const int64_t r0 = UNPACK ? H->nreq_dir[0] : 0, r1 = r0 + H->nreq_dir[UNPACK];
    const int64_t t_begin = ordered ? (UNPACK ? H->nslots_dir[0] : 0) : (UNPACK ? H->ntiles_dir[0] : 0);
    const int64_t t_end = t_begin + (ordered ? H->nslots_dir[UNPACK] : H->ntiles_dir[UNPACK]);
    int64_t t;
    if (POLICY != 1) {
        t = t_begin + blockIdx.x;
    } else {
        if (threadIdx.x == 0) s_t = t_begin + (int64_t)atomicAdd(counter, 1ull);
        __syncthreads();
        t = uniform64(s_t);
    }
    while (t < t_end) {
        const int64_t tile = ordered ? (int64_t)order[t] : t;  // -1: an empty slot
        if (tile >= 0) {
            // request holding the tile: last r with tile0[r] <= tile
            int64_t lo = r0, hi = r1 - 1;
            while (lo < hi) {
                int64_t mid = (lo + hi + 1) >> 1;
                if (tile0[mid] <= tile) lo = mid; else hi = mid - 1;
            }
            const ReqDesc &D = R[lo];
            const DevLayout &L = const_layout(D.lay);
            XferArgs A;
            A.typed = D.typed;
            A.packed = D.packed;
            A.off = D.off;
            A.nbytes = D.nbytes;
            A.head = D.head;
            A.nchunks = D.nchunks;
            const int64_t T = D.tc;
            A.tile_chunks = T;
            A.elem1 = D.elem1;
            A.keep = (int32_t)H->keep_packed;
            int64_t c0 = (tile - tile0[lo]) * T;
            int64_t cend = c0 + T < D.nchunks ? c0 + T : D.nchunks;
            run_tile<UNPACK, BODY>(L, A, D.body, D.kind, c0, cend, lds_dyn, D);
        }
        if (POLICY == 2) break;
        if (POLICY == 0) {
            t += gridDim.x;
        } else {
            __syncthreads();
            if (threadIdx.x == 0) s_t = t_begin + (int64_t)atomicAdd(counter, 1ull);
            __syncthreads();
            t = uniform64(s_t);
        }
    }
}

}  // namespace mdt

namespace mdt {

// Launch one direction's kernel, compiled for the tile bodies `body` names
// (a set of BODY_* bits).  Defined in batch_variants.hip, compiled once per pair.
template <int POLICY, int UNPACK>
void launch_batch_dir(dim3 grid, size_t lds, hipStream_t s, const BatchHeader *H, const ReqDesc *R,
                      const int64_t *tile0, const int32_t *order, unsigned long long *counter, int body);
#define MDT_BATCH_DIR(P, U)                                                                                \
    template <>                                                                                            \
    void launch_batch_dir<P, U>(dim3 grid, size_t lds, hipStream_t s, const BatchHeader *H, const ReqDesc *R, \
                                const int64_t *tile0, const int32_t *order, unsigned long long *counter, int body);
MDT_BATCH_DIR(0, 0)
MDT_BATCH_DIR(0, 1)
MDT_BATCH_DIR(1, 0)
MDT_BATCH_DIR(1, 1)
MDT_BATCH_DIR(2, 0)
MDT_BATCH_DIR(2, 1)
#undef MDT_BATCH_DIR

// one direction: a kernel with only the body the direction needs, else one
// with all (copies run with the pack direction only)
template <int POLICY, int UNPACK>
void launch_batch_dir_impl(dim3 grid, size_t lds, hipStream_t s, const BatchHeader *H, const ReqDesc *R,
                           const int64_t *tile0, const int32_t *order, unsigned long long *counter, int body)
{
#define MDT_LAUNCH(BODY) hipLaunchKernelGGL((batch_kernel<POLICY, UNPACK, BODY>), grid, dim3(256), lds, s, H, R, \
                                            tile0, order, counter)
    if (!UNPACK && (body & BODY_RELAY)) {
        if ((body & ~(BODY_RELAY | BODY_CHUNK)) == 0) MDT_LAUNCH(UNPACK ? BODY_ALL : (BODY_RELAY | BODY_CHUNK));
        else MDT_LAUNCH(UNPACK ? BODY_ALL : (BODY_RELAY | BODY_ALL | BODY_COPY));
    } else if (!UNPACK && body == BODY_COPY) MDT_LAUNCH(UNPACK ? BODY_ALL : BODY_COPY);
    else if (!UNPACK && (body & BODY_COPY)) MDT_LAUNCH(UNPACK ? BODY_ALL : (BODY_ALL | BODY_COPY));
    else if (body == BODY_DENSE) MDT_LAUNCH(BODY_DENSE);
    else if (body == BODY_RUNS) MDT_LAUNCH(BODY_RUNS);
    else if (!UNPACK && body == (BODY_CHUNK | BODY_CACHED)) MDT_LAUNCH(UNPACK ? BODY_ALL : (BODY_CHUNK | BODY_CACHED));
    else if (body == BODY_CHUNK) MDT_LAUNCH(BODY_CHUNK);
    else MDT_LAUNCH(BODY_ALL);
#undef MDT_LAUNCH
}

}  // namespace mdt
