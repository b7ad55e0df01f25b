// device.h -- launch interface of the gfx950 kernels (host side).
#pragma once

#include <hip/hip_runtime_api.h>

#include "core.h"

namespace mdt {

// One pack or unpack over bytes [off, off + nbytes) of a packed stream.
struct XferArgs {
    const uint8_t *typed;  // origin of the typed (non-contiguous) buffer
    uint8_t *packed;       // first packed byte (stream position off)
    int64_t off;           // stream position of packed[0]
    int64_t nbytes;        // packed bytes moved
    int64_t head;          // packed & 15: the chunk grid is 16-byte aligned
    int64_t nchunks;       // 16-byte chunks covering [packed, packed + nbytes)
    int64_t tile_chunks;   // chunks per workgroup tile (0: default)
    int32_t elem1;         // off + nbytes <= element size: only element 0 is touched
    int32_t keep;          // pack: cached stores for the packed output (see KEEP_PACKED_MAX)
};

// A pack whose output is at most this large stores it with ordinary (cached)
// stores, so whatever consumes it next (an unpack, a send) reads it from the
// 256 MiB Infinity Cache; larger outputs stream past the caches.  Measured on
// the halo step (61 MiB packed, unpacked right after): 105.4 -> 97.3 us per
// step, though the pack alone takes longer (45.6 -> 53.1 us).
constexpr int64_t KEEP_PACKED_MAX = (int64_t)128 << 20;

// One typed copy: bytes [off, off + nbytes) of the source stream go to the
// same positions of the destination stream.  Chunk c covers stream bytes
// [off + 16c, off + 16c + 16).
struct CopyArgs {
    const uint8_t *src;    // origin of the source buffer
    uint8_t *dst;          // origin of the destination buffer
    int64_t off;           // first stream position copied
    int64_t nbytes;        // bytes copied
    int64_t nchunks;       // ceil(nbytes / 16)
    int32_t src_elem1;     // off + nbytes <= source element size
    int32_t dst_elem1;     // off + nbytes <= destination element size
};

XferArgs make_args(const void *typed, void *packed, int64_t off, int64_t nbytes);
int launch_copy(const DevLayout &Ls, const DevLayout &Ld, const CopyArgs &A, hipStream_t s);
int launch_xfer(const DevLayout &L, const XferArgs &A, bool unpack, hipStream_t s);
// sc: the count form's segments (NULL or count 1: one element)
int launch_flatten(Compiled *c, DeviceTables *d, int64_t off, int64_t m, mdt_iov *out, const void *base,
                   hipStream_t s, const SegCount *sc = nullptr);
int64_t default_tile_chunks(int64_t nchunks);
// the dense record path applies to this request
bool use_dense(const DevLayout &L, const XferArgs &A, bool unpack);
// the run-table kernel (LDS-cached group slice) applies
bool use_runs(const DevLayout &L);

}  // namespace mdt
