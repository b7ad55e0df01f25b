// core.h -- host-side internals of libmdt: type nodes, the layout IR that
// commit compiles them to, and the lowered (device-ready) form.
#pragma once

#include <atomic>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mdt.h"
#include "layout_dev.h"

namespace mdt {

enum Kind {
    K_BASIC,
    K_CONTIG,
    K_VECTOR,
    K_HVECTOR,
    K_INDEXED,
    K_HINDEXED,
    K_STRUCT,
    K_SUBARRAY,
    K_RESIZED,
    K_DUP
};

// ---- layout IR -------------------------------------------------------
struct Loop {
    int64_t cnt, stride;
    bool operator==(const Loop &o) const { return cnt == o.cnt && stride == o.stride; }
};
struct Run {
    int64_t off, len;
    bool operator==(const Run &o) const { return off == o.off && len == o.len; }
};
// A regular body: loops (outer to inner) over a list of leaf runs.
struct Shape {
    std::vector<Loop> loops;
    std::vector<Run> leaf;
    bool varlen = false;     // one run at offset 0, as long as its group
    bool implicit0 = false;  // loops[0].cnt = group length / span of loop 0
    bool operator==(const Shape &o) const
    {
        if (varlen != o.varlen || implicit0 != o.implicit0 || leaf != o.leaf) return false;
        if (loops.size() != o.loops.size()) return false;
        for (size_t l = 0; l < loops.size(); l++) {
            if (loops[l].stride != o.loops[l].stride) return false;
            if (!(implicit0 && l == 0) && loops[l].cnt != o.loops[l].cnt) return false;
        }
        return true;
    }
};
struct Group {
    int64_t disp, len;
    int32_t shape;
};
// outer loops x groups x (shape loops x leaf)
struct Layout {
    std::vector<Loop> outer;
    std::vector<Group> groups;
    std::vector<Shape> shapes;
    int64_t size = 0;
};
using LayoutP = std::shared_ptr<const Layout>;

// ---- committed state -------------------------------------------------
struct DeviceTables {
    int device = -1;
    DevLayout lay{};          // with device pointers
    DevLayout *d_lay = nullptr;  // device copy of `lay`
    std::vector<void *> allocs;
    // segment table (only for layouts whose runs can merge)
    mdt_iov *d_segs = nullptr;
};

struct Compiled {
    LayoutP layout;
    // lowered host form
    DevLayout host{};  // host pointers into the vectors below
    std::vector<int64_t> gdisp, gpre, grpre;
    std::vector<int32_t> gshape, gdir;
    std::vector<DevShape> shapes;
    std::vector<std::vector<int64_t>> leaf_store;  // big leaf arrays (off, len, pre per shape)
    std::vector<uint32_t> rec_ptab, rec_ttab;       // record-view byte tables
    std::vector<uint32_t> rec_ctab, rec_dtab;       // record-view chunk (pack) and dword (unpack) tables
    bool rec_count1_only = false;                   // record view holds for element 0 only
    int64_t nruns = 0;
    bool merge_free = true;
    // segment table for layouts that are not merge-free, built on demand
    std::once_flag seg_once;
    int seg_status = MDT_SUCCESS;
    std::vector<int64_t> seg_addr, seg_len, seg_pre;
    // overlap classification, computed on demand
    std::mutex ov_mu;
    int64_t ov_checked_count = -1;  // largest count proven overlap-free
    bool self_disjoint = false;     // structural: one element has no overlap
    int64_t true_lb = 0, true_ub = 0, extent = 0;
    // device uploads (one per device)
    std::mutex dev_mu;
    std::vector<std::unique_ptr<DeviceTables>> dev;
    ~Compiled();
};

struct TypeNode {
    uint32_t magic = 0x6d647421u;
    std::atomic<int> refs{1};
    Kind kind = K_BASIC;
    bool predefined = false;
    // constructor arguments (deep copies)
    int64_t n = 0, bl = 0, stride = 0;
    std::vector<int64_t> bls, disps;
    std::vector<TypeNode *> kids;  // referenced children
    int nd = 0, order = 0;
    std::vector<int64_t> sizes, subs, starts;
    int64_t rlb = 0, rext = 0;
    // the constructor call as made (type envelope and contents): combiner,
    // integer and address arguments, and the child types, which this
    // node's own children keep alive
    int combiner = 0;
    std::vector<int64_t> c_ints, c_addrs;
    std::vector<TypeNode *> c_types;
    // attributes
    int64_t size = 0, lb = 0, ub = 0, tlb = 0, tub = 0, align = 1;
    bool expl = false;
    // compilation
    std::mutex mu;
    LayoutP layout;                      // memoized layout IR
    std::shared_ptr<Compiled> comp;      // set by commit
    std::atomic<bool> committed{false};
    int64_t extent() const { return ub - lb; }
};

// types.cpp
bool valid_type(const TypeNode *t);
void retain(TypeNode *t);
void release(TypeNode *t);

// compile.cpp
int compile_layout(TypeNode *t, LayoutP *out);
int commit_type(TypeNode *t);
int host_iov_len(TypeNode *t, int64_t max_bytes, int64_t *n, int64_t *bytes);
int host_iov(TypeNode *t, int64_t off, mdt_iov *iov, int64_t m, int64_t *actual);
int check_unpack_overlap(Compiled *c, int64_t count);  // MDT_SUCCESS or MDT_ERR_OVERLAP / NO_MEM
// segments of count consecutive elements (compile.cpp)
struct SegCount {
    Compiled *C;
    int64_t count, extent, size;
    int64_t n;      // segments of one element
    bool merge;     // an element's last segment merges with the next element's first
    int64_t total;  // segments of the count form
};
int element_segments(TypeNode *t, SegCount *sc, int64_t count);
void seg_of(const SegCount &sc, int64_t j, int64_t *addr, int64_t *len);
void seg_count_at(const SegCount &sc, int64_t g, int64_t *addr, int64_t *len);
int host_iov_len_count(TypeNode *t, int64_t count, int64_t max_bytes, int64_t *n, int64_t *bytes);
int host_iov_count(TypeNode *t, int64_t count, int64_t off, mdt_iov *iov, int64_t m, int64_t *actual);
int build_segment_table(Compiled *c);

// device.hip
int device_tables(Compiled *c, DeviceTables **out);  // upload on first use per device
// the tables already resident on the current device; MDT_ERR_STATE if none (no upload)
int device_tables_resident(Compiled *c, DeviceTables **out);
void free_device_tables(DeviceTables *d);
void set_hip_error(int e);

// limits
constexpr int64_t MAX_GROUPS = (int64_t)1 << 25;
constexpr int64_t MAX_SEG_TABLE = (int64_t)1 << 26;
constexpr int64_t MAX_OVERLAP_RUNS = (int64_t)1 << 26;

}  // namespace mdt
