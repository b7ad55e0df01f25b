// types.cpp -- type constructors and their attributes, in closed form.
//
// Each constructor places copies of its child at a set of byte shifts (the
// MPI constructor definitions the Derived Datatypes section relies on).  The
// attributes of the result follow from the range of those shifts and the
// child's attributes, so they cost O(blocks), never O(entries):
//   lb / ub            min / max over placed copies of shift + lb(c) / ub(c)
//   true_lb / true_ub  the same over copies of children that hold bytes
//   size               (number of copies) x size(c)
// struct pads its extent to its largest member alignment unless a member
// has explicit bounds; subarray and resized set explicit bounds.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "core.h"
#include "trace.h"

namespace mdt {

namespace {

bool add_ok(int64_t a, int64_t b, int64_t *r) { return !__builtin_add_overflow(a, b, r); }
bool mul_ok(int64_t a, int64_t b, int64_t *r) { return !__builtin_mul_overflow(a, b, r); }

// min / max of i*step for 0 <= i < cnt (cnt >= 1)
bool lin_range(int64_t cnt, int64_t step, int64_t *lo, int64_t *hi)
{
    int64_t v;
    if (!mul_ok(cnt - 1, step, &v)) return false;
    *lo = std::min<int64_t>(0, v);
    *hi = std::max<int64_t>(0, v);
    return true;
}

struct Acc {
    bool placed = false, data = false, ovf = false;
    int64_t lb = 0, ub = 0, tlb = 0, tub = 0, size = 0, align = 1;
    bool expl = false;
    // copies of child c whose shifts span [slo, shi]; ncopies of them
    void add(const TypeNode *c, int64_t slo, int64_t shi, int64_t ncopies)
    {
        if (ncopies <= 0) return;
        int64_t v;
        if (!add_ok(slo, c->lb, &v)) { ovf = true; return; }
        lb = placed ? std::min(lb, v) : v;
        if (!add_ok(shi, c->ub, &v)) { ovf = true; return; }
        ub = placed ? std::max(ub, v) : v;
        placed = true;
        if (c->size > 0) {
            if (!add_ok(slo, c->tlb, &v)) { ovf = true; return; }
            tlb = data ? std::min(tlb, v) : v;
            if (!add_ok(shi, c->tub, &v)) { ovf = true; return; }
            tub = data ? std::max(tub, v) : v;
            data = true;
        }
        int64_t s;
        if (!mul_ok(ncopies, c->size, &s) || !add_ok(size, s, &size)) { ovf = true; return; }
        align = std::max(align, c->align);
        expl = expl || c->expl;
    }
};

int finish(TypeNode *t, Acc &A)
{
    if (A.ovf) return MDT_ERR_ARG;
    t->size = A.size;
    t->align = A.align;
    t->expl = A.expl;
    t->lb = A.placed ? A.lb : 0;
    t->ub = A.placed ? A.ub : 0;
    t->tlb = A.data ? A.tlb : 0;
    t->tub = A.data ? A.tub : 0;
    int64_t e;
    if (t->kind == K_STRUCT && !A.expl && A.placed) {
        int64_t ext;
        if (__builtin_sub_overflow(t->ub, t->lb, &ext)) return MDT_ERR_ARG;
        if (ext > 0 && ext % A.align != 0 && !add_ok(t->ub, A.align - ext % A.align, &t->ub)) return MDT_ERR_ARG;
    }
    if (__builtin_sub_overflow(t->ub, t->lb, &e) || __builtin_sub_overflow(t->tub, t->tlb, &e)) return MDT_ERR_ARG;
    return MDT_SUCCESS;
}

TypeNode *new_node(Kind k) { return new (std::nothrow) TypeNode(); }

int attach(TypeNode *t, TypeNode *c)
{
    retain(c);
    t->kids.push_back(c);
    return MDT_SUCCESS;
}

int done(TypeNode *t, Acc &A, mdt_type *out)
{
    int rc = finish(t, A);
    if (rc != MDT_SUCCESS) {
        release(t);
        return rc;
    }
    *out = reinterpret_cast<mdt_type>(t);
    return MDT_SUCCESS;
}

TypeNode *as_node(mdt_type t) { return reinterpret_cast<TypeNode *>(t); }

// predefined types
struct Predef {
    TypeNode nodes[MDT_NUM_BASIC];
    Predef()
    {
        static const int64_t sz[MDT_NUM_BASIC] = {1, 1, 1, 1, 2, 2, 4, 4, 4, 4, 8, 8, 8};
        for (int i = 0; i < MDT_NUM_BASIC; i++) {
            TypeNode &n = nodes[i];
            n.kind = K_BASIC;
            n.predefined = true;
            n.refs = 1 << 30;
            n.size = sz[i];
            n.lb = 0;
            n.ub = sz[i];
            n.tlb = 0;
            n.tub = sz[i];
            n.align = sz[i];
        }
    }
};
Predef &predef()
{
    static Predef p;
    return p;
}

}  // namespace

bool valid_type(const TypeNode *t) { return t && t->magic == 0x6d647421u && t->refs.load() > 0; }

void retain(TypeNode *t)
{
    if (!t->predefined) t->refs.fetch_add(1);
}

void release(TypeNode *t)
{
    if (t->predefined) return;
    if (t->refs.fetch_sub(1) == 1) {
        for (TypeNode *c : t->kids) release(c);
        t->magic = 0;
        delete t;
    }
}

}  // namespace mdt

using namespace mdt;

// Record the constructor call (type envelope and contents) on the type it
// returned.
static int record(int rc, mdt_type *out, int combiner, std::vector<int64_t> ints, std::vector<int64_t> addrs,
                  std::vector<mdt_type> types)
{
    if (rc != MDT_SUCCESS) return rc;
    TypeNode *t = as_node(*out);
    try {
        t->combiner = combiner;
        t->c_ints = std::move(ints);
        t->c_addrs = std::move(addrs);
        t->c_types.clear();
        for (mdt_type x : types) t->c_types.push_back(as_node(x));
    } catch (...) {
        mdt_type_free(out);
        return MDT_ERR_NO_MEM;
    }
    return rc;
}

static std::vector<int64_t> cat(std::vector<int64_t> a, const int64_t *b, int64_t n)
{
    if (n > 0 && b) a.insert(a.end(), b, b + n);
    return a;
}

static std::vector<int64_t> darray_ints(int size, int rank, int nd, const int64_t *gsizes, const int *distribs,
                                        const int *dargs, const int *psizes, int order)
{
    std::vector<int64_t> v = cat({size, rank, nd}, gsizes, nd);
    for (int k = 0; k < nd; k++) v.push_back(distribs[k]);
    for (int k = 0; k < nd; k++) v.push_back(dargs[k]);
    for (int k = 0; k < nd; k++) v.push_back(psizes[k]);
    v.push_back(order);
    return v;
}

#define CHECK_TYPE(t)                                         \
    do {                                                      \
        if (!valid_type(reinterpret_cast<TypeNode *>(t))) return MDT_ERR_TYPE; \
    } while (0)

extern "C" {

MDT_API mdt_type mdt_basic(int code)
{
    if (code < 0 || code >= MDT_NUM_BASIC) return MDT_TYPE_NULL;
    return reinterpret_cast<mdt_type>(&predef().nodes[code]);
}

MDT_API int mdt_type_contiguous(mdt_count n, mdt_type old, mdt_type *out)
{
    CHECK_TYPE(old);
    if (!out || n < 0) return MDT_ERR_ARG;
    TypeNode *c = as_node(old);
    TypeNode *t = new_node(K_CONTIG);
    if (!t) return MDT_ERR_NO_MEM;
    t->kind = K_CONTIG;
    t->n = n;
    attach(t, c);
    Acc A;
    if (n > 0) {
        int64_t lo, hi;
        if (!lin_range(n, c->extent(), &lo, &hi)) A.ovf = true;
        else A.add(c, lo, hi, n);
    }
    return record(done(t, A, out), out, MDT_COMBINER_CONTIGUOUS, {n}, {}, {old});
}

static int make_hvec(Kind k, int64_t n, int64_t bl, int64_t stride_bytes, int64_t stride_elems, TypeNode *c,
                     mdt_type *out)
{
    TypeNode *t = new_node(k);
    if (!t) return MDT_ERR_NO_MEM;
    t->kind = k;
    t->n = n;
    t->bl = bl;
    t->stride = k == K_VECTOR ? stride_elems : stride_bytes;
    attach(t, c);
    Acc A;
    if (n > 0 && bl > 0) {
        int64_t lo1 = 0, hi1 = 0, lo2, hi2, v;
        if (n > 1) {
            if (k == K_VECTOR) {
                // (i*stride + j) * E: i*stride*E over i, checked as ((n-1)*stride)*E
                if (!mul_ok(n - 1, stride_elems, &v) || !mul_ok(v, c->extent(), &v)) A.ovf = true;
                lo1 = std::min<int64_t>(0, v);
                hi1 = std::max<int64_t>(0, v);
            } else if (!lin_range(n, stride_bytes, &lo1, &hi1)) {
                A.ovf = true;
            }
        }
        if (!lin_range(bl, c->extent(), &lo2, &hi2)) A.ovf = true;
        int64_t lo, hi, cnt;
        if (!add_ok(lo1, lo2, &lo) || !add_ok(hi1, hi2, &hi) || !mul_ok(n, bl, &cnt)) A.ovf = true;
        if (!A.ovf) A.add(c, lo, hi, cnt);
    }
    return done(t, A, out);
}

MDT_API int mdt_type_vector(mdt_count n, mdt_count bl, mdt_count stride, mdt_type old, mdt_type *out)
{
    CHECK_TYPE(old);
    if (!out || n < 0 || bl < 0) return MDT_ERR_ARG;
    return record(make_hvec(K_VECTOR, n, bl, 0, stride, as_node(old), out), out, MDT_COMBINER_VECTOR, {n, bl, stride},
                  {}, {old});
}

MDT_API int mdt_type_create_hvector(mdt_count n, mdt_count bl, mdt_aint stride_bytes, mdt_type old,
                                    mdt_type *out)
{
    CHECK_TYPE(old);
    if (!out || n < 0 || bl < 0) return MDT_ERR_ARG;
    return record(make_hvec(K_HVECTOR, n, bl, stride_bytes, 0, as_node(old), out), out, MDT_COMBINER_HVECTOR, {n, bl},
                  {stride_bytes}, {old});
}

// indexed family: block i holds bl[i] copies starting at disp[i] (elements
// of E for indexed, bytes for hindexed).
static int make_idx(Kind k, int64_t n, const int64_t *bl, int64_t bl1, const int64_t *disp, bool in_extents,
                    TypeNode *c, mdt_type *out)
{
    if (!out || n < 0 || (n > 0 && !disp)) return MDT_ERR_ARG;
    if (bl) {
        for (int64_t i = 0; i < n; i++)
            if (bl[i] < 0) return MDT_ERR_ARG;
    } else if (bl1 < 0) {
        return MDT_ERR_ARG;
    }
    TypeNode *t = new_node(k);
    if (!t) return MDT_ERR_NO_MEM;
    t->kind = k;
    t->n = n;
    try {
        t->bls.resize(n);
        t->disps.resize(n);
    } catch (...) {
        delete t;
        return MDT_ERR_NO_MEM;
    }
    const int64_t E = c->extent();
    Acc A;
    for (int64_t i = 0; i < n && !A.ovf; i++) {
        int64_t b = bl ? bl[i] : bl1;
        int64_t d = disp[i];
        t->bls[i] = b;
        t->disps[i] = 0;
        if (b == 0) continue;
        if (in_extents && !mul_ok(d, E, &d)) {
            A.ovf = true;
            break;
        }
        t->disps[i] = d;  // stored in bytes
        int64_t lo, hi;
        if (!lin_range(b, E, &lo, &hi) || !add_ok(lo, d, &lo) || !add_ok(hi, d, &hi)) {
            A.ovf = true;
            break;
        }
        A.add(c, lo, hi, b);
    }
    t->kind = K_HINDEXED;  // indexed is stored as hindexed with byte displacements
    attach(t, c);
    return done(t, A, out);
}

MDT_API int mdt_type_indexed(mdt_count n, const mdt_count bl[], const mdt_count disp[], mdt_type old,
                             mdt_type *out)
{
    CHECK_TYPE(old);
    if (n > 0 && !bl) return MDT_ERR_ARG;
    return record(make_idx(K_INDEXED, n, bl, 0, disp, true, as_node(old), out), out, MDT_COMBINER_INDEXED,
                  cat(cat({n}, bl, n), disp, n), {}, {old});
}

MDT_API int mdt_type_create_hindexed(mdt_count n, const mdt_count bl[], const mdt_aint disp[], mdt_type old,
                                     mdt_type *out)
{
    CHECK_TYPE(old);
    if (n > 0 && !bl) return MDT_ERR_ARG;
    return record(make_idx(K_HINDEXED, n, bl, 0, disp, false, as_node(old), out), out, MDT_COMBINER_HINDEXED,
                  cat({n}, bl, n), cat({}, disp, n), {old});
}

MDT_API int mdt_type_create_indexed_block(mdt_count n, mdt_count bl, const mdt_count disp[], mdt_type old,
                                          mdt_type *out)
{
    CHECK_TYPE(old);
    return record(make_idx(K_INDEXED, n, nullptr, bl, disp, true, as_node(old), out), out,
                  MDT_COMBINER_INDEXED_BLOCK, cat({n, bl}, disp, n), {}, {old});
}

MDT_API int mdt_type_create_hindexed_block(mdt_count n, mdt_count bl, const mdt_aint disp[], mdt_type old,
                                           mdt_type *out)
{
    CHECK_TYPE(old);
    return record(make_idx(K_HINDEXED, n, nullptr, bl, disp, false, as_node(old), out), out,
                  MDT_COMBINER_HINDEXED_BLOCK, {n, bl}, cat({}, disp, n), {old});
}

MDT_API int mdt_type_create_struct(mdt_count n, const mdt_count bl[], const mdt_aint disp[],
                                   const mdt_type types[], mdt_type *out)
{
    if (!out || n < 0 || (n > 0 && (!bl || !disp || !types))) return MDT_ERR_ARG;
    for (int64_t i = 0; i < n; i++) {
        if (!valid_type(as_node(types[i]))) return MDT_ERR_TYPE;
        if (bl[i] < 0) return MDT_ERR_ARG;
    }
    TypeNode *t = new_node(K_STRUCT);
    if (!t) return MDT_ERR_NO_MEM;
    t->kind = K_STRUCT;
    t->n = n;
    Acc A;
    try {
        t->bls.assign(bl, bl + n);
        t->disps.assign(disp, disp + n);
    } catch (...) {
        delete t;
        return MDT_ERR_NO_MEM;
    }
    for (int64_t i = 0; i < n; i++) {
        TypeNode *c = as_node(types[i]);
        attach(t, c);
        if (bl[i] == 0 || A.ovf) continue;
        int64_t lo, hi;
        if (!lin_range(bl[i], c->extent(), &lo, &hi) || !add_ok(lo, disp[i], &lo) || !add_ok(hi, disp[i], &hi)) {
            A.ovf = true;
            continue;
        }
        A.add(c, lo, hi, bl[i]);
    }
    return record(done(t, A, out), out, MDT_COMBINER_STRUCT, cat({n}, bl, n), cat({}, disp, n),
                  std::vector<mdt_type>(types, types + n));
}

MDT_API int mdt_type_create_subarray(int ndims, const mdt_count sizes[], const mdt_count subsizes[],
                                     const mdt_count starts[], int order, mdt_type old, mdt_type *out)
{
    CHECK_TYPE(old);
    if (!out || ndims < 1 || ndims > 32 || !sizes || !subsizes || !starts) return MDT_ERR_ARG;
    if (order != MDT_ORDER_C && order != MDT_ORDER_FORTRAN) return MDT_ERR_ARG;
    for (int k = 0; k < ndims; k++) {
        if (sizes[k] < 1 || subsizes[k] < 0 || starts[k] < 0) return MDT_ERR_ARG;
        if (subsizes[k] > sizes[k] || starts[k] > sizes[k] - subsizes[k]) return MDT_ERR_ARG;
    }
    TypeNode *c = as_node(old);
    TypeNode *t = new_node(K_SUBARRAY);
    if (!t) return MDT_ERR_NO_MEM;
    t->kind = K_SUBARRAY;
    t->nd = ndims;
    t->order = order;
    t->sizes.assign(sizes, sizes + ndims);
    t->subs.assign(subsizes, subsizes + ndims);
    t->starts.assign(starts, starts + ndims);
    attach(t, c);
    Acc A;
    // linear index multiplier of each dimension
    int64_t total = 1;
    std::vector<int64_t> mult(ndims);
    bool empty = false;
    for (int i = 0; i < ndims; i++) {
        int k = order == MDT_ORDER_C ? ndims - 1 - i : i;
        mult[k] = total;
        if (!mul_ok(total, sizes[k], &total)) A.ovf = true;
        if (subsizes[k] == 0) empty = true;
    }
    int64_t E = c->extent(), ub;
    if (!mul_ok(total, E, &ub)) A.ovf = true;
    if (!empty && !A.ovf) {
        int64_t lmin = 0, lmax = 0, v, cnt = 1;
        for (int k = 0; k < ndims && !A.ovf; k++) {
            if (!mul_ok(starts[k], mult[k], &v) || !add_ok(lmin, v, &lmin)) A.ovf = true;
            if (!mul_ok(starts[k] + subsizes[k] - 1, mult[k], &v) || !add_ok(lmax, v, &lmax)) A.ovf = true;
            if (!mul_ok(cnt, subsizes[k], &cnt)) A.ovf = true;
        }
        int64_t a, b;
        if (!A.ovf && mul_ok(lmin, E, &a) && mul_ok(lmax, E, &b)) A.add(c, std::min(a, b), std::max(a, b), cnt);
        else A.ovf = true;
    }
    if (!A.ovf) {
        // bounds of the whole array, explicit
        A.placed = true;
        A.lb = 0;
        A.ub = ub;
        A.expl = true;
    }
    std::vector<int64_t> ci = cat(cat(cat({ndims}, sizes, ndims), subsizes, ndims), starts, ndims);
    ci.push_back(order);
    return record(done(t, A, out), out, MDT_COMBINER_SUBARRAY, std::move(ci), {}, {old});
}

MDT_API int mdt_type_create_resized(mdt_type old, mdt_aint lb, mdt_aint extent, mdt_type *out)
{
    CHECK_TYPE(old);
    if (!out) return MDT_ERR_ARG;
    TypeNode *c = as_node(old);
    TypeNode *t = new_node(K_RESIZED);
    if (!t) return MDT_ERR_NO_MEM;
    t->kind = K_RESIZED;
    t->rlb = lb;
    t->rext = extent;
    attach(t, c);
    Acc A;
    A.add(c, 0, 0, 1);
    int64_t ub;
    if (!add_ok(lb, extent, &ub)) A.ovf = true;
    A.lb = lb;
    A.ub = ub;
    A.placed = true;
    A.expl = true;
    return record(done(t, A, out), out, MDT_COMBINER_RESIZED, {}, {lb, extent}, {old});
}

MDT_API int mdt_type_dup(mdt_type old, mdt_type *out)
{
    CHECK_TYPE(old);
    if (!out) return MDT_ERR_ARG;
    TypeNode *c = as_node(old);
    TypeNode *t = new_node(K_DUP);
    if (!t) return MDT_ERR_NO_MEM;
    t->kind = K_DUP;
    attach(t, c);
    Acc A;
    A.add(c, 0, 0, 1);
    A.align = c->align;
    A.expl = c->expl;
    int rc = done(t, A, out);
    if (rc == MDT_SUCCESS) {
        // a dup keeps the bounds of its child exactly
        TypeNode *d = as_node(*out);
        d->lb = c->lb;
        d->ub = c->ub;
    }
    return record(rc, out, MDT_COMBINER_DUP, {}, {}, {old});
}

// Distributed array: the indices each dimension owns are a list of blocks
// (one for a block or undistributed dimension, several for a cyclic one).
// With one block per dimension the result is the subarray of those blocks;
// otherwise it is built one dimension at a time, fastest first: an hindexed
// of the blocks over the faster dimensions' type, resized to the whole
// dimension, so the next dimension steps over complete hyperplanes.
MDT_API int mdt_type_create_darray(int size, int rank, int ndims, const mdt_count gsizes[], const int distribs[],
                                   const int dargs[], const int psizes[], int order, mdt_type old, mdt_type *out)
{
    CHECK_TYPE(old);
    if (!out || ndims < 1 || ndims > 32 || !gsizes || !distribs || !dargs || !psizes) return MDT_ERR_ARG;
    if (order != MDT_ORDER_C && order != MDT_ORDER_FORTRAN) return MDT_ERR_ARG;
    if (size < 1 || rank < 0 || rank >= size) return MDT_ERR_ARG;
    int64_t nproc = 1;
    for (int k = 0; k < ndims; k++) {
        if (gsizes[k] < 1 || psizes[k] < 1 || !mul_ok(nproc, psizes[k], &nproc)) return MDT_ERR_ARG;
    }
    if (nproc != size) return MDT_ERR_ARG;
    // grid coordinates: ranks are row-major over the process grid
    std::vector<int64_t> coord(ndims);
    for (int k = ndims - 1, r = rank; k >= 0; k--) {
        coord[k] = r % psizes[k];
        r /= psizes[k];
    }
    // owned indices of every dimension as equally spaced blocks: `count`
    // blocks of `len` indices, the first at `first`, `step` apart, the last
    // one `last` long (0 blocks when the coordinate owns nothing)
    struct Blocks {
        int64_t first = 0, len = 0, step = 0, count = 0, last = 0;
    };
    std::vector<Blocks> blocks(ndims);
    bool single = true;
    for (int k = 0; k < ndims; k++) {
        const int64_t g = gsizes[k], P = psizes[k], c = coord[k];
        const int d = dargs[k];
        Blocks &B = blocks[k];
        if (d != MDT_DISTRIBUTE_DFLT_DARG && d < 1) return MDT_ERR_ARG;
        if (distribs[k] == MDT_DISTRIBUTE_NONE || (distribs[k] == MDT_DISTRIBUTE_CYCLIC && P == 1)) {
            if (distribs[k] == MDT_DISTRIBUTE_NONE && P != 1) return MDT_ERR_ARG;
            B = {0, g, g, 1, g};  // the whole dimension
        } else if (distribs[k] == MDT_DISTRIBUTE_BLOCK) {
            const int64_t b = d == MDT_DISTRIBUTE_DFLT_DARG ? (g + P - 1) / P : d;
            int64_t cover;
            if (!mul_ok(b, P, &cover) || cover < g) return MDT_ERR_ARG;
            const int64_t st = c * b;
            if (st < g) B = {st, std::min(b, g - st), b, 1, std::min(b, g - st)};
        } else if (distribs[k] == MDT_DISTRIBUTE_CYCLIC) {
            const int64_t b = d == MDT_DISTRIBUTE_DFLT_DARG ? 1 : d;
            int64_t step, first;
            if (!mul_ok(b, P, &step) || !mul_ok(c, b, &first)) return MDT_ERR_ARG;
            if (first < g) {
                const int64_t count = (g - first + step - 1) / step;
                const int64_t last_start = first + (count - 1) * step;
                B = {first, b, step, count, std::min(b, g - last_start)};
                if (count == 1) B.len = B.last;
            }
        } else {
            return MDT_ERR_ARG;
        }
        single = single && B.count <= 1;
    }
    if (single) {
        std::vector<mdt_count> sub(ndims), st(ndims);
        for (int k = 0; k < ndims; k++) {
            sub[k] = blocks[k].count ? blocks[k].len : 0;
            st[k] = blocks[k].count ? blocks[k].first : 0;
        }
        return record(mdt_type_create_subarray(ndims, gsizes, sub.data(), st.data(), order, old, out), out,
                      MDT_COMBINER_DARRAY, darray_ints(size, rank, ndims, gsizes, distribs, dargs, psizes, order), {},
                      {old});
    }
    // fastest dimension first; cur holds a reference the loop owns (old is
    // borrowed until the first step replaces it).  A dimension's full
    // blocks are equally spaced, so they are one strided vector (the layout
    // compiler turns it into a loop), placed at the first block; a shorter
    // last block follows it as a second struct member.
    mdt_type cur = old;
    bool owned = false;
    int64_t E = as_node(old)->extent();
    int rc = MDT_SUCCESS;
    for (int i = 0; i < ndims && rc == MDT_SUCCESS; i++) {
        const int k = order == MDT_ORDER_C ? ndims - 1 - i : i;
        const Blocks &B = blocks[k];
        int64_t span;
        if (!mul_ok(gsizes[k], E, &span)) rc = MDT_ERR_ARG;
        mdt_type placed = MDT_TYPE_NULL;  // the dimension's owned blocks of cur, at their displacements
        int64_t d0 = 0;
        if (rc == MDT_SUCCESS && !mul_ok(B.first, E, &d0)) rc = MDT_ERR_ARG;
        if (rc == MDT_SUCCESS && B.count <= 1) {
            mdt_count bl = B.count ? B.len : 0;
            rc = mdt_type_create_hindexed(B.count, &bl, &d0, cur, &placed);
        } else if (rc == MDT_SUCCESS) {
            const int64_t nfull = B.last == B.len ? B.count : B.count - 1;
            int64_t stride, dt;
            if (!mul_ok(B.step, E, &stride) || !mul_ok(B.first + (B.count - 1) * B.step, E, &dt)) rc = MDT_ERR_ARG;
            mdt_type vec = MDT_TYPE_NULL;
            if (rc == MDT_SUCCESS) rc = mdt_type_create_hvector(nfull, B.len, stride, cur, &vec);
            if (rc == MDT_SUCCESS && nfull == B.count) {
                mdt_count one = 1;
                rc = mdt_type_create_hindexed(1, &one, &d0, vec, &placed);
            } else if (rc == MDT_SUCCESS) {
                mdt_count bl2[2] = {1, B.last};
                mdt_aint disp2[2] = {d0, dt};
                mdt_type kids[2] = {vec, cur};
                rc = mdt_type_create_struct(2, bl2, disp2, kids, &placed);
            }
            if (vec) mdt_type_free(&vec);
        }
        mdt_type r = MDT_TYPE_NULL;
        if (rc == MDT_SUCCESS) rc = mdt_type_create_resized(placed, 0, span, &r);
        if (placed) mdt_type_free(&placed);
        if (owned) mdt_type_free(&cur);
        cur = r;
        owned = true;
        E = span;
    }
    if (rc != MDT_SUCCESS) {
        if (owned && cur) mdt_type_free(&cur);
        return rc;
    }
    *out = cur;
    return record(MDT_SUCCESS, out, MDT_COMBINER_DARRAY,
                  darray_ints(size, rank, ndims, gsizes, distribs, dargs, psizes, order), {}, {old});
}

MDT_API int mdt_type_get_envelope(mdt_type t, mdt_count *num_integers, mdt_count *num_addresses,
                                  mdt_count *num_datatypes, int *combiner)
{
    CHECK_TYPE(t);
    if (!num_integers || !num_addresses || !num_datatypes || !combiner) return MDT_ERR_ARG;
    const TypeNode *n = as_node(t);
    *num_integers = (mdt_count)n->c_ints.size();
    *num_addresses = (mdt_count)n->c_addrs.size();
    *num_datatypes = (mdt_count)n->c_types.size();
    *combiner = n->predefined ? MDT_COMBINER_NAMED : n->combiner;
    return MDT_SUCCESS;
}

MDT_API int mdt_type_get_contents(mdt_type t, mdt_count max_integers, mdt_count max_addresses,
                                  mdt_count max_datatypes, mdt_count integers[], mdt_aint addresses[],
                                  mdt_type datatypes[])
{
    CHECK_TYPE(t);
    const TypeNode *n = as_node(t);
    const int64_t ni = (int64_t)n->c_ints.size(), na = (int64_t)n->c_addrs.size(), nt = (int64_t)n->c_types.size();
    if (n->predefined || max_integers < ni || max_addresses < na || max_datatypes < nt) return MDT_ERR_ARG;
    if ((ni && !integers) || (na && !addresses) || (nt && !datatypes)) return MDT_ERR_ARG;
    std::copy(n->c_ints.begin(), n->c_ints.end(), integers);
    std::copy(n->c_addrs.begin(), n->c_addrs.end(), addresses);
    for (int64_t i = 0; i < nt; i++) {
        TypeNode *c = n->c_types[(size_t)i];
        if (!c->predefined) retain(c);
        datatypes[i] = reinterpret_cast<mdt_type>(c);
    }
    return MDT_SUCCESS;
}

MDT_API int mdt_type_commit(mdt_type *t)
{
    mdt::TraceRange trace_("mdt_type_commit");
    if (!t) return MDT_ERR_ARG;
    CHECK_TYPE(*t);
    return commit_type(as_node(*t));
}

MDT_API int mdt_type_free(mdt_type *t)
{
    if (!t) return MDT_ERR_ARG;
    CHECK_TYPE(*t);
    TypeNode *n = as_node(*t);
    if (n->predefined) return MDT_ERR_TYPE;
    release(n);
    *t = MDT_TYPE_NULL;
    return MDT_SUCCESS;
}

MDT_API int mdt_type_layout_info(mdt_type t, mdt_layout_info *out)
{
    CHECK_TYPE(t);
    if (!out) return MDT_ERR_ARG;
    TypeNode *n = as_node(t);
    if (!n->committed.load() || !n->comp) return MDT_ERR_TYPE;
    const Compiled &C = *n->comp;
    const DevLayout &L = C.host;
    std::memset(out, 0, sizeof *out);
    out->kind = L.kind;
    out->groups = L.kind == KIND_MULTI ? L.G : (L.kind == KIND_EMPTY ? 0 : 1);
    out->runs = L.nruns;
    out->records = L.rec.on;
    if (L.rec.on) {
        out->record_bytes = L.rec.U;
        out->record_stride = L.rec.X;
        out->pack_table = L.rec.ctab ? 2 : 1;
        out->unpack_table = L.rec.dtab ? 2 : (L.rec.ttab ? 1 : 0);
    }
    int64_t b = (int64_t)(C.shapes.size() * sizeof(DevShape) + sizeof(DevLayout));
    for (auto &v : C.leaf_store) b += (int64_t)(v.size() * sizeof(int64_t));
    b += (int64_t)((C.gdisp.size() + C.gpre.size() + C.grpre.size()) * sizeof(int64_t));
    b += (int64_t)((C.gshape.size() + C.gdir.size()) * sizeof(int32_t));
    b += (int64_t)((C.rec_ptab.size() + C.rec_ttab.size() + C.rec_ctab.size() + C.rec_dtab.size()) * sizeof(uint32_t));
    out->device_bytes = b;
    return MDT_SUCCESS;
}

MDT_API int mdt_type_size(mdt_type t, mdt_count *size)
{
    CHECK_TYPE(t);
    if (!size) return MDT_ERR_ARG;
    *size = as_node(t)->size;
    return MDT_SUCCESS;
}

MDT_API int mdt_type_get_extent(mdt_type t, mdt_aint *lb, mdt_aint *extent)
{
    CHECK_TYPE(t);
    if (!lb || !extent) return MDT_ERR_ARG;
    *lb = as_node(t)->lb;
    *extent = as_node(t)->extent();
    return MDT_SUCCESS;
}

MDT_API int mdt_type_get_true_extent(mdt_type t, mdt_aint *true_lb, mdt_aint *true_extent)
{
    CHECK_TYPE(t);
    if (!true_lb || !true_extent) return MDT_ERR_ARG;
    *true_lb = as_node(t)->tlb;
    *true_extent = as_node(t)->tub - as_node(t)->tlb;
    return MDT_SUCCESS;
}

MDT_API int mdt_type_iov_len(mdt_type t, mdt_count max_iov_bytes, mdt_count *iov_len,
                             mdt_count *actual_iov_bytes)
{
    CHECK_TYPE(t);
    if (!iov_len || !actual_iov_bytes || max_iov_bytes < -1) return MDT_ERR_ARG;
    TypeNode *n = as_node(t);
    if (!n->committed.load() && !n->predefined) return MDT_ERR_TYPE;
    return host_iov_len(n, max_iov_bytes, iov_len, actual_iov_bytes);
}

MDT_API int mdt_type_iov(mdt_type t, mdt_count iov_offset, mdt_iov *iov, mdt_count max_iov_len,
                         mdt_count *actual_iov_len)
{
    CHECK_TYPE(t);
    if (!actual_iov_len || iov_offset < 0 || max_iov_len < 0 || (max_iov_len > 0 && !iov)) return MDT_ERR_ARG;
    TypeNode *n = as_node(t);
    if (!n->committed.load() && !n->predefined) return MDT_ERR_TYPE;
    return host_iov(n, iov_offset, iov, max_iov_len, actual_iov_len);
}

MDT_API int mdt_type_iov_len_count(mdt_type t, mdt_count count, mdt_count max_iov_bytes, mdt_count *iov_len,
                                   mdt_count *actual_iov_bytes)
{
    CHECK_TYPE(t);
    if (!iov_len || !actual_iov_bytes || max_iov_bytes < -1 || count < 0) return MDT_ERR_ARG;
    TypeNode *n = as_node(t);
    if (!n->committed.load() && !n->predefined) return MDT_ERR_TYPE;
    return host_iov_len_count(n, count, max_iov_bytes, iov_len, actual_iov_bytes);
}

MDT_API int mdt_type_iov_count(mdt_type t, mdt_count count, mdt_count iov_offset, mdt_iov *iov,
                               mdt_count max_iov_len, mdt_count *actual_iov_len)
{
    CHECK_TYPE(t);
    if (!actual_iov_len || count < 0 || iov_offset < 0 || max_iov_len < 0 || (max_iov_len > 0 && !iov))
        return MDT_ERR_ARG;
    TypeNode *n = as_node(t);
    if (!n->committed.load() && !n->predefined) return MDT_ERR_TYPE;
    return host_iov_count(n, count, iov_offset, iov, max_iov_len, actual_iov_len);
}

MDT_API const char *mdt_error_string(int code)
{
    switch (code) {
    case MDT_SUCCESS: return "success";
    case MDT_ERR_ARG: return "invalid argument";
    case MDT_ERR_TYPE: return "invalid, freed or uncommitted datatype";
    case MDT_ERR_COUNT: return "count out of range for the datatype";
    case MDT_ERR_TRUNCATE: return "packed input longer than the remaining stream";
    case MDT_ERR_OVERLAP: return "unpack target layout overlaps itself";
    case MDT_ERR_NO_MEM: return "out of memory or size limit";
    case MDT_ERR_HIP: return "HIP runtime error";
    case MDT_ERR_AGAIN: return "admission budget full, try again";
    case MDT_ERR_STATE: return "invalid state for this call";
    default: return "unknown error";
    }
}

MDT_API int mdt_version(void) { return 100; }

}  // extern "C"
