// host_sanitize.cpp -- the host halves of the library and the oracle under
// AddressSanitizer and UndefinedBehaviorSanitizer.
//
// The library's constructors and layout compiler (types.cpp, compile.cpp,
// compiled unchanged with the host compiler; host_stub.cpp stands in for
// the device tables) and the oracle (oracle/oracle.c) build the same
// seeded random types side by side -- every constructor (distributed
// arrays with invalid arguments among them), nested, with
// negative strides and displacements, zero block lengths, empty subarrays,
// resized bounds -- and must agree on the attributes, on every segment of
// one element and of 0, 2 and 3 elements, on iov_len at a spread of
// budgets, and on the address of every packed byte as the kernels' seek
// (locate on the layout program, run on the host) finds it.  Envelope/contents, layout info and the error paths run too, and
// the oracle packs and unpacks every type at random offsets and budgets.
// Any out-of-bounds access, leak or undefined behaviour ends the run with
// the sanitizer's report.  Then 2000 types with huge counts, strides,
// displacements and bounds (library only) must build or fail with
// MDT_ERR_ARG, and commit and every query must return a result or an error,
// with no undefined behaviour.  Prints "host sanitize ok".
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "core.h"  // the layout compiler's own entry points (overlap check)
#include "mdt.h"

extern "C" {
#include "oracle.h"
}

#define CHECK(cond)                                                                        \
    do {                                                                                   \
        if (!(cond)) {                                                                     \
            std::fprintf(stderr, "%s:%d: check failed: %s (type %d)\n", __FILE__, __LINE__, #cond, g_case); \
            std::exit(1);                                                                  \
        }                                                                                  \
    } while (0)

namespace {

int g_case = -1;
std::mt19937_64 g_rng(20240219);
int64_t g_derived = 0, g_segments = 0, g_packs = 0, g_located = 0;

int64_t rnd(int64_t lo, int64_t hi) { return lo + (int64_t)(g_rng() % (uint64_t)(hi - lo + 1)); }

struct Pair {
    mdt_type m = nullptr;
    orc_type *o = nullptr;
};

void release(Pair &p)
{
    if (p.m && p.m != mdt_basic(MDT_CODE_BYTE) && p.m != mdt_basic(MDT_CODE_INT16) &&
        p.m != mdt_basic(MDT_CODE_INT32) && p.m != mdt_basic(MDT_CODE_DOUBLE))
        CHECK(mdt_type_free(&p.m) == MDT_SUCCESS && p.m == nullptr);
    if (p.o) orc_release(p.o);
    p.m = nullptr;
    p.o = nullptr;
}

Pair basic()
{
    static const int codes[] = {MDT_CODE_BYTE, MDT_CODE_INT16, MDT_CODE_INT32, MDT_CODE_DOUBLE};
    static const int64_t sizes[] = {1, 2, 4, 8};
    const int k = (int)rnd(0, 3);
    Pair p;
    p.m = mdt_basic(codes[k]);
    int e = 0;
    p.o = orc_basic(sizes[k], &e);
    CHECK(p.m && p.o);
    return p;
}

// A random type of nesting depth <= depth, built by both sides.
Pair gen(int depth)
{
    if (depth == 0 || rnd(0, 4) == 0) return basic();
    const int k = (int)rnd(0, 11);
    Pair c = k == 8 ? Pair{} : gen(depth - 1);
    Pair p;
    int e = 0, rm = MDT_SUCCESS;
    switch (k) {
    case 0: {
        const int64_t n = rnd(0, 4);
        rm = mdt_type_contiguous(n, c.m, &p.m);
        p.o = orc_contiguous(n, c.o, &e);
        break;
    }
    case 1: {
        const int64_t n = rnd(0, 4), bl = rnd(0, 3), st = rnd(-4, 5);
        rm = mdt_type_vector(n, bl, st, c.m, &p.m);
        p.o = orc_vector(n, bl, st, c.o, &e);
        break;
    }
    case 2: {
        const int64_t n = rnd(0, 4), bl = rnd(0, 3), st = rnd(-40, 40);
        rm = mdt_type_create_hvector(n, bl, st, c.m, &p.m);
        p.o = orc_hvector(n, bl, st, c.o, &e);
        break;
    }
    case 3:
    case 4: {
        const int64_t n = rnd(0, 4);
        std::vector<int64_t> bl((size_t)n + 1), d((size_t)n + 1);
        for (int64_t i = 0; i < n; i++) {
            bl[(size_t)i] = rnd(0, 3);
            d[(size_t)i] = k == 3 ? rnd(-6, 10) : rnd(-50, 60);
        }
        if (k == 3) {
            rm = mdt_type_indexed(n, bl.data(), d.data(), c.m, &p.m);
            p.o = orc_indexed(n, bl.data(), d.data(), c.o, &e);
        } else {
            rm = mdt_type_create_hindexed(n, bl.data(), d.data(), c.m, &p.m);
            p.o = orc_hindexed(n, bl.data(), d.data(), c.o, &e);
        }
        break;
    }
    case 5:
    case 6: {
        const int64_t n = rnd(0, 4), bl = rnd(0, 3);
        std::vector<int64_t> d((size_t)n + 1);
        for (int64_t i = 0; i < n; i++) d[(size_t)i] = k == 5 ? rnd(-6, 10) : rnd(-50, 60);
        if (k == 5) {
            rm = mdt_type_create_indexed_block(n, bl, d.data(), c.m, &p.m);
            p.o = orc_indexed_block(n, bl, d.data(), c.o, &e);
        } else {
            rm = mdt_type_create_hindexed_block(n, bl, d.data(), c.m, &p.m);
            p.o = orc_hindexed_block(n, bl, d.data(), c.o, &e);
        }
        break;
    }
    case 7: {
        const int nd = (int)rnd(1, 3);
        int64_t sz[3], sub[3], st[3];
        for (int i = 0; i < nd; i++) {
            sz[i] = rnd(1, 4);
            sub[i] = rnd(0, sz[i]);
            st[i] = rnd(0, sz[i] - sub[i]);
        }
        const int order = (int)rnd(0, 1);
        rm = mdt_type_create_subarray(nd, sz, sub, st, order ? MDT_ORDER_FORTRAN : MDT_ORDER_C, c.m, &p.m);
        p.o = orc_subarray(nd, sz, sub, st, order ? ORC_ORDER_FORTRAN : ORC_ORDER_C, c.o, &e);
        break;
    }
    case 8: {
        const int64_t n = rnd(1, 3);
        std::vector<Pair> kids;
        std::vector<int64_t> bl, d;
        std::vector<mdt_type> km;
        std::vector<orc_type *> ko;
        for (int64_t i = 0; i < n; i++) {
            kids.push_back(gen(depth - 1));
            bl.push_back(rnd(0, 2));
            d.push_back(rnd(-30, 50));
            km.push_back(kids.back().m);
            ko.push_back(kids.back().o);
        }
        rm = mdt_type_create_struct(n, bl.data(), d.data(), km.data(), &p.m);
        p.o = orc_struct(n, bl.data(), d.data(), ko.data(), &e);
        for (auto &x : kids) release(x);
        break;
    }
    case 9: {
        const int64_t lb = rnd(-16, 16), ext = rnd(1, 64);
        rm = mdt_type_create_resized(c.m, lb, ext, &p.m);
        p.o = orc_resized(c.o, lb, ext, &e);
        break;
    }
    case 11: {
        // a distributed array: every distribution, default and explicit
        // arguments (some of them invalid: both sides must refuse those)
        const int nd = (int)rnd(1, 3);
        int64_t gs[3];
        int dist[3], darg[3], ps[3], size = 1;
        for (int i = 0; i < nd; i++) {
            gs[i] = rnd(1, 9);
            dist[i] = (int)rnd(0, 2);
            ps[i] = dist[i] == MDT_DISTRIBUTE_NONE && rnd(0, 7) ? 1 : (int)rnd(1, 3);
            darg[i] = rnd(0, 2) == 0 ? MDT_DISTRIBUTE_DFLT_DARG : (int)rnd(0, 5);
            size *= ps[i];
        }
        const int rank = (int)rnd(0, size);  // size itself: an invalid rank
        const int order = (int)rnd(0, 1);
        rm = mdt_type_create_darray(size, rank, nd, gs, dist, darg, ps, order ? MDT_ORDER_FORTRAN : MDT_ORDER_C, c.m,
                                    &p.m);
        p.o = orc_darray(size, rank, nd, gs, dist, darg, ps, order ? ORC_ORDER_FORTRAN : ORC_ORDER_C, c.o, &e);
        break;
    }
    default:
        rm = mdt_type_dup(c.m, &p.m);
        p.o = orc_dup(c.o, &e);
        break;
    }
    release(c);  // both sides deep-copy or reference what they need
    CHECK((rm == MDT_SUCCESS) == (p.o != nullptr));
    if (rm != MDT_SUCCESS) return basic();
    return p;
}

// The constructor tree of t (from its envelope and contents), for a report.
void describe(mdt_type t, int indent)
{
    mdt_count ni = 0, na = 0, nt = 0;
    int comb = -1;
    if (mdt_type_get_envelope(t, &ni, &na, &nt, &comb) != MDT_SUCCESS) return;
    mdt_count size = 0;
    mdt_aint lb = 0, ext = 0;
    mdt_type_size(t, &size);
    mdt_type_get_extent(t, &lb, &ext);
    std::fprintf(stderr, "%*scombiner %d size %lld lb %lld extent %lld", indent, "", comb, (long long)size,
                 (long long)lb, (long long)ext);
    if (comb == MDT_COMBINER_NAMED) {
        std::fprintf(stderr, "\n");
        return;
    }
    std::vector<mdt_count> ints((size_t)ni + 1);
    std::vector<mdt_aint> addrs((size_t)na + 1);
    std::vector<mdt_type> types((size_t)nt + 1);
    mdt_type_get_contents(t, ni, na, nt, ints.data(), addrs.data(), types.data());
    std::fprintf(stderr, " ints");
    for (mdt_count i = 0; i < ni; i++) std::fprintf(stderr, " %lld", (long long)ints[(size_t)i]);
    std::fprintf(stderr, " addrs");
    for (mdt_count i = 0; i < na; i++) std::fprintf(stderr, " %lld", (long long)addrs[(size_t)i]);
    std::fprintf(stderr, "\n");
    for (mdt_count i = 0; i < nt; i++) {
        describe(types[(size_t)i], indent + 2);
        mdt_count a1, a2, a3;
        int c2 = -1;
        if (mdt_type_get_envelope(types[(size_t)i], &a1, &a2, &a3, &c2) == MDT_SUCCESS && c2 != MDT_COMBINER_NAMED)
            mdt_type_free(&types[(size_t)i]);
    }
}

void check_segments(const Pair &p, int64_t count)
{
    int64_t nseg = 0;
    CHECK(orc_num_segments_count(p.o, count, &nseg) == ORC_OK);
    mdt_count n = -1, bytes = -1;
    CHECK(mdt_type_iov_len_count(p.m, count, -1, &n, &bytes) == MDT_SUCCESS);
    CHECK(n == nseg);
    std::vector<mdt_iov> iov((size_t)nseg + 1);
    std::vector<int64_t> ob((size_t)nseg + 1), ol((size_t)nseg + 1);
    mdt_count got = -1;
    int64_t ogot = -1;
    CHECK(mdt_type_iov_count(p.m, count, 0, iov.data(), nseg, &got) == MDT_SUCCESS && got == nseg);
    CHECK(orc_iov_count(p.o, count, 0, ob.data(), ol.data(), nseg, &ogot) == ORC_OK && ogot == nseg);
    int64_t sum = 0;
    for (int64_t i = 0; i < nseg; i++) {
        const int64_t b = (int64_t)(intptr_t)iov[(size_t)i].iov_base, l = iov[(size_t)i].iov_len;
        if (b != ob[(size_t)i] || l != ol[(size_t)i]) {
            std::fprintf(stderr, "count %lld segment %lld of %lld: library (%lld, %lld), oracle (%lld, %lld)\n",
                         (long long)count, (long long)i, (long long)nseg, (long long)b, (long long)l,
                         (long long)ob[(size_t)i], (long long)ol[(size_t)i]);
            describe(p.m, 0);
        }
        CHECK(b == ob[(size_t)i] && l == ol[(size_t)i]);
        sum += ol[(size_t)i];
    }
    CHECK(sum == bytes);
    g_segments += nseg;
    // the seek the kernels use (locate on the layout program, here on the
    // host): every packed byte of the count-fold stream maps to the address
    // the oracle's segments give it, inside a run that ends within them
    if (bytes > 0 && bytes <= 65536) {
        const mdt::DevLayout &L = reinterpret_cast<mdt::TypeNode *>(p.m)->comp->host;
        int64_t pos = 0;
        for (int64_t i = 0; i < nseg; i++) {
            for (int64_t q = 0; q < ol[(size_t)i]; q++) {
                const mdt::Loc l = mdt::locate_any(L, (uint64_t)(pos + q));
                // (the contiguous kind reports its one run as unbounded)
                const bool rem_ok = L.kind == mdt::KIND_CONTIG || (l.rem >= 1 && l.rem <= ol[(size_t)i] - q);
                if (l.addr != ob[(size_t)i] + q || !rem_ok)
                    std::fprintf(stderr, "count %lld byte %lld: located (%lld, %lld), oracle address %lld, segment end %lld\n",
                                 (long long)count, (long long)(pos + q), (long long)l.addr, (long long)l.rem,
                                 (long long)(ob[(size_t)i] + q), (long long)(ob[(size_t)i] + ol[(size_t)i]));
                CHECK(l.addr == ob[(size_t)i] + q && rem_ok);
            }
            pos += ol[(size_t)i];
        }
        g_located += pos;
    }
    // budgets: whole segments only, and their bytes
    const int64_t budgets[] = {0, 1, 7, bytes / 3, bytes / 2, bytes - 1, bytes};
    for (int64_t b : budgets) {
        if (b < 0) continue;
        mdt_count k1 = -1, a1 = -1;
        int64_t k2 = -1, a2 = -1;
        CHECK(mdt_type_iov_len_count(p.m, count, b, &k1, &a1) == MDT_SUCCESS);
        CHECK(orc_iov_len_count(p.o, count, b, &k2, &a2) == ORC_OK);
        CHECK(k1 == k2 && a1 == a2);
    }
    // a slice from the middle
    if (nseg > 2) {
        const int64_t off = nseg / 2, m = nseg - off + 2;
        std::vector<mdt_iov> s((size_t)m);
        CHECK(mdt_type_iov_count(p.m, count, off, s.data(), m, &got) == MDT_SUCCESS && got == nseg - off);
        CHECK((int64_t)(intptr_t)s[0].iov_base == ob[(size_t)off] && s[0].iov_len == ol[(size_t)off]);
    }
}

void check_pair(const Pair &p)
{
    int64_t a[8];
    CHECK(orc_attrs(p.o, a) == ORC_OK);
    mdt_count size = -1;
    mdt_aint lb = 0, ext = 0, tlb = 0, text = 0;
    CHECK(mdt_type_size(p.m, &size) == MDT_SUCCESS && size == a[0]);
    CHECK(mdt_type_get_extent(p.m, &lb, &ext) == MDT_SUCCESS && lb == a[1] && ext == a[2] - a[1]);
    CHECK(mdt_type_get_true_extent(p.m, &tlb, &text) == MDT_SUCCESS);
    if (size > 0) CHECK(tlb == a[3] && text == a[4] - a[3]);
    // queries need a committed type
    mdt_count n = 0, bytes = 0;
    const bool basic_type = mdt_type_iov_len(p.m, -1, &n, &bytes) == MDT_SUCCESS;
    mdt_type t = p.m;
    if (!basic_type) {
        CHECK(mdt_type_iov_len(p.m, -1, &n, &bytes) == MDT_ERR_TYPE);
        CHECK(mdt_type_commit(&t) == MDT_SUCCESS && t == p.m);
        CHECK(mdt_type_commit(&t) == MDT_SUCCESS);  // twice is fine
    }
    for (int64_t count : {1, 0, 2, 3}) check_segments(p, count);
    mdt_layout_info li{};
    CHECK(mdt_type_layout_info(p.m, &li) == MDT_SUCCESS);
    // envelope and contents, and the types they hand back
    mdt_count ni = -1, na = -1, nt = -1;
    int comb = -1;
    CHECK(mdt_type_get_envelope(p.m, &ni, &na, &nt, &comb) == MDT_SUCCESS);
    if (comb != MDT_COMBINER_NAMED) {
        g_derived++;
        std::vector<mdt_count> ints((size_t)ni + 1);
        std::vector<mdt_aint> addrs((size_t)na + 1);
        std::vector<mdt_type> types((size_t)nt + 1);
        if (ni > 0) CHECK(mdt_type_get_contents(p.m, ni - 1, na, nt, ints.data(), addrs.data(), types.data()) ==
                          MDT_ERR_ARG);
        CHECK(mdt_type_get_contents(p.m, ni, na, nt, ints.data(), addrs.data(), types.data()) == MDT_SUCCESS);
        for (mdt_count i = 0; i < nt; i++) {
            mdt_count a1, a2, a3;
            int c2 = -1;
            CHECK(mdt_type_get_envelope(types[(size_t)i], &a1, &a2, &a3, &c2) == MDT_SUCCESS);
            if (c2 != MDT_COMBINER_NAMED) CHECK(mdt_type_free(&types[(size_t)i]) == MDT_SUCCESS);
        }
    }
    // the oracle moves the bytes: pack at random ranges, unpack back
    for (int64_t count : {1, 3}) {
        if (size == 0) break;
        const int64_t span_lo = std::min(a[3], a[3] + (count - 1) * (a[2] - a[1]));
        const int64_t span_hi = std::max(a[4], a[4] + (count - 1) * (a[2] - a[1]));
        const int64_t nbuf = span_hi - span_lo + 8;
        std::vector<uint8_t> buf((size_t)nbuf), back((size_t)nbuf, 0);
        for (auto &x : buf) x = (uint8_t)g_rng();
        uint8_t *origin = buf.data() - span_lo + 4;
        const int64_t total = count * size;
        std::vector<uint8_t> full((size_t)total + 1), part((size_t)total + 1);
        int64_t got = -1;
        CHECK(orc_pack(origin, count, p.o, 0, full.data(), -1, &got) == ORC_OK && got == total);
        const int64_t off = rnd(0, total), mx = rnd(-1, total);
        CHECK(orc_pack(origin, count, p.o, off, part.data(), mx, &got) == ORC_OK);
        CHECK(got == std::max<int64_t>(0, mx < 0 ? total - off : std::min(mx, total - off)));
        CHECK(std::memcmp(part.data(), full.data() + off, (size_t)got) == 0);
        int64_t got2 = -1;
        CHECK(orc_pack_mt(origin, count, p.o, 0, part.data(), -1, &got2, 2) == ORC_OK && got2 == total);
        CHECK(std::memcmp(part.data(), full.data(), (size_t)total) == 0);
        uint8_t *borigin = back.data() - span_lo + 4;
        const int ru = orc_unpack(full.data(), total, borigin, count, p.o, 0, &got2);
        g_packs++;
        CHECK(ru == ORC_OK || ru == ORC_ERR_OVERLAP);
        // the library's unpack overlap verdict is the oracle's
        mdt::TypeNode *tn = reinterpret_cast<mdt::TypeNode *>(p.m);
        const int rl = mdt::check_unpack_overlap(tn->comp.get(), count);
        CHECK((rl == MDT_ERR_OVERLAP) == (ru == ORC_ERR_OVERLAP) && (rl == MDT_SUCCESS || rl == MDT_ERR_OVERLAP));
    }
}

// ---- extreme parameters (library only: the oracle enumerates copies one by
// one and is not meant for 2^40-element types) ------------------------------

int64_t big_count()
{
    static const int64_t v[] = {0, 1, 2, 3, 1000, 1000000, (int64_t)1 << 31, (int64_t)1 << 40, (int64_t)1 << 62};
    return v[rnd(0, 8)];
}

int64_t big_signed()
{
    static const int64_t v[] = {1, 7, (int64_t)1 << 20, (int64_t)1 << 40, (int64_t)1 << 61, INT64_MAX / 3};
    const int64_t x = v[rnd(0, 5)];
    return rnd(0, 1) ? x : -x;
}

int64_t cnt_or_big(int64_t lo, int64_t hi) { return rnd(0, 2) == 0 ? big_count() : rnd(lo, hi); }
int64_t off_or_big(int64_t lo, int64_t hi) { return rnd(0, 2) == 0 ? big_signed() : rnd(lo, hi); }

// A random type whose counts, strides, displacements, sizes and bounds are
// often huge; every constructor must either build it or return an error
// (MDT_ERR_ARG on overflow), with no undefined behaviour on the way.
mdt_type gen_extreme(int depth)
{
    static const int codes[] = {MDT_CODE_BYTE, MDT_CODE_INT16, MDT_CODE_INT32, MDT_CODE_DOUBLE};
    if (depth == 0 || rnd(0, 4) == 0) return mdt_basic(codes[rnd(0, 3)]);
    const int k = (int)rnd(0, 9);
    mdt_type c = gen_extreme(depth - 1), t = nullptr;
    int rc = MDT_SUCCESS;
    int64_t bl[3], d[3];
    for (int i = 0; i < 3; i++) {
        bl[i] = cnt_or_big(0, 3);
        d[i] = off_or_big(-50, 60);
    }
    switch (k) {
    case 0: rc = mdt_type_contiguous(cnt_or_big(0, 4), c, &t); break;
    case 1: rc = mdt_type_vector(cnt_or_big(0, 4), cnt_or_big(0, 3), off_or_big(-4, 5), c, &t); break;
    case 2: rc = mdt_type_create_hvector(cnt_or_big(0, 4), cnt_or_big(0, 3), off_or_big(-40, 40), c, &t); break;
    case 3: rc = mdt_type_indexed(3, bl, d, c, &t); break;
    case 4: rc = mdt_type_create_hindexed(3, bl, d, c, &t); break;
    case 5: rc = mdt_type_create_hindexed_block(3, cnt_or_big(0, 3), d, c, &t); break;
    case 6: {
        mdt_type kids[3] = {c, gen_extreme(depth - 1), mdt_basic(codes[rnd(0, 3)])};
        rc = mdt_type_create_struct(3, bl, d, kids, &t);
        mdt_count a, b, n;
        int comb = -1;
        if (mdt_type_get_envelope(kids[1], &a, &b, &n, &comb) == MDT_SUCCESS && comb != MDT_COMBINER_NAMED)
            mdt_type_free(&kids[1]);
        break;
    }
    case 7: {
        const int nd = (int)rnd(1, 3);
        mdt_count sz[3], sub[3], st[3];
        for (int i = 0; i < nd; i++) {
            sz[i] = rnd(0, 1) ? ((int64_t)1 << rnd(10, 40)) : rnd(1, 4);
            sub[i] = rnd(0, 1) ? sz[i] : rnd(0, std::min<int64_t>(sz[i], 4));
            st[i] = rnd(0, std::min<int64_t>(sz[i] - sub[i], 3));
        }
        rc = mdt_type_create_subarray(nd, sz, sub, st, rnd(0, 1) ? MDT_ORDER_FORTRAN : MDT_ORDER_C, c, &t);
        break;
    }
    case 8: rc = mdt_type_create_resized(c, off_or_big(-16, 16), rnd(0, 1) ? big_count() : rnd(1, 64), &t); break;
    default: rc = mdt_type_dup(c, &t); break;
    }
    mdt_count a, b, n;
    int comb = -1;
    if (mdt_type_get_envelope(c, &a, &b, &n, &comb) == MDT_SUCCESS && comb != MDT_COMBINER_NAMED) mdt_type_free(&c);
    CHECK(rc == MDT_SUCCESS || rc == MDT_ERR_ARG);
    CHECK((rc == MDT_SUCCESS) == (t != nullptr));
    return rc == MDT_SUCCESS ? t : mdt_basic(codes[rnd(0, 3)]);
}

int64_t g_extreme_built = 0, g_extreme_committed = 0;

// Everything a caller can ask of such a type, on the host.
void check_extreme(mdt_type t)
{
    mdt_count size = -1, ni, na, nt;
    mdt_aint lb, ext, tlb, text;
    int comb = -1;
    CHECK(mdt_type_size(t, &size) == MDT_SUCCESS && size >= 0);
    CHECK(mdt_type_get_extent(t, &lb, &ext) == MDT_SUCCESS);
    CHECK(mdt_type_get_true_extent(t, &tlb, &text) == MDT_SUCCESS && text >= 0);
    CHECK(mdt_type_get_envelope(t, &ni, &na, &nt, &comb) == MDT_SUCCESS);
    if (comb == MDT_COMBINER_NAMED) return;
    g_extreme_built++;
    mdt_type c = t;
    const int rc = mdt_type_commit(&c);
    CHECK(rc == MDT_SUCCESS || rc == MDT_ERR_NO_MEM || rc == MDT_ERR_ARG || rc == MDT_ERR_COUNT);
    if (rc != MDT_SUCCESS) return;
    g_extreme_committed++;
    mdt_layout_info li{};
    CHECK(mdt_type_layout_info(t, &li) == MDT_SUCCESS);
    for (mdt_count budget : {(mdt_count)-1, (mdt_count)0, (mdt_count)1, (mdt_count)4096, size / 2, size}) {
        mdt_count k = -1, bytes = -1;
        const int r = mdt_type_iov_len(t, budget, &k, &bytes);
        CHECK(r == MDT_SUCCESS || r == MDT_ERR_NO_MEM || r == MDT_ERR_COUNT);
        if (r == MDT_SUCCESS) CHECK(k >= 0 && bytes >= 0 && bytes <= size);
    }
    mdt::TypeNode *tn = reinterpret_cast<mdt::TypeNode *>(t);
    // the exact overlap check sorts every run: keep to types of few runs here
    for (int64_t count : {(int64_t)1, (int64_t)2, (int64_t)1 << 40, (int64_t)1 << 62}) {
        if (li.runs > 65536) break;
        const int ro = mdt::check_unpack_overlap(tn->comp.get(), count);
        CHECK(ro == MDT_SUCCESS || ro == MDT_ERR_OVERLAP || ro == MDT_ERR_NO_MEM || ro == MDT_ERR_COUNT);
    }
    mdt_iov iov[4];
    mdt_count got = -1;
    int r = mdt_type_iov(t, 0, iov, 4, &got);
    CHECK(r == MDT_SUCCESS || r == MDT_ERR_NO_MEM || r == MDT_ERR_COUNT);
    r = mdt_type_iov(t, (mdt_count)1 << 40, iov, 4, &got);
    CHECK(r == MDT_SUCCESS || r == MDT_ERR_NO_MEM || r == MDT_ERR_COUNT);
    for (mdt_count count : {(mdt_count)2, (mdt_count)1 << 20, (mdt_count)1 << 62}) {
        mdt_count k = -1, bytes = -1;
        r = mdt_type_iov_len_count(t, count, 4096, &k, &bytes);
        CHECK(r == MDT_SUCCESS || r == MDT_ERR_NO_MEM || r == MDT_ERR_COUNT);
        r = mdt_type_iov_count(t, count, 3, iov, 4, &got);
        CHECK(r == MDT_SUCCESS || r == MDT_ERR_NO_MEM || r == MDT_ERR_COUNT);
    }
}

void check_errors()
{
    mdt_type t = nullptr;
    const mdt_type D = mdt_basic(MDT_CODE_DOUBLE);
    CHECK(mdt_type_vector(-1, 1, 1, D, &t) == MDT_ERR_ARG && t == nullptr);
    CHECK(mdt_type_contiguous(2, nullptr, &t) == MDT_ERR_TYPE);
    const mdt_count sz[2] = {4, 4}, sub[2] = {3, 3}, st[2] = {2, 0};
    CHECK(mdt_type_create_subarray(2, sz, sub, st, MDT_ORDER_C, D, &t) == MDT_ERR_ARG);
    CHECK(mdt_type_contiguous((mdt_count)1 << 61, D, &t) == MDT_ERR_ARG);  // 2^64 bytes: overflow
    CHECK(mdt_type_contiguous(3, D, &t) == MDT_SUCCESS);
    CHECK(mdt_type_free(&t) == MDT_SUCCESS && t == nullptr);
    CHECK(mdt_type_free(&t) != MDT_SUCCESS);
    CHECK(mdt_type_iov_len_count(D, -1, -1, nullptr, nullptr) != MDT_SUCCESS);
    // regressions: a zero-count vector of copies of a 2^62 extent commits
    // (its parts are never laid out), and the overlap check of a type with
    // no bytes returns at once for 2^40 elements
    mdt_type big = nullptr, empty = nullptr, e2 = nullptr;
    CHECK(mdt_type_create_resized(D, -((int64_t)1 << 61), (int64_t)1 << 62, &big) == MDT_SUCCESS);
    CHECK(mdt_type_create_hvector(0, 3, 1 << 20, big, &empty) == MDT_SUCCESS);
    CHECK(mdt_type_commit(&empty) == MDT_SUCCESS);
    CHECK(mdt_type_create_resized(empty, 0, 8, &e2) == MDT_SUCCESS && mdt_type_commit(&e2) == MDT_SUCCESS);
    CHECK(mdt::check_unpack_overlap(reinterpret_cast<mdt::TypeNode *>(e2)->comp.get(), (int64_t)1 << 40) ==
          MDT_SUCCESS);
    CHECK(mdt_type_free(&e2) == MDT_SUCCESS && mdt_type_free(&empty) == MDT_SUCCESS && mdt_type_free(&big) == MDT_SUCCESS);
    int e = 0;
    CHECK(orc_vector(-1, 1, 1, nullptr, &e) == nullptr);
}

}  // namespace

int main()
{
    check_errors();
    for (g_case = 0; g_case < 2000; g_case++) {
        Pair p = gen((int)rnd(1, 3));
        check_pair(p);
        release(p);
    }
    for (g_case = 0; g_case < 2000; g_case++) {
        mdt_type t = gen_extreme((int)rnd(1, 3));
        check_extreme(t);
        mdt_count a, b, n;
        int comb = -1;
        if (mdt_type_get_envelope(t, &a, &b, &n, &comb) == MDT_SUCCESS && comb != MDT_COMBINER_NAMED)
            CHECK(mdt_type_free(&t) == MDT_SUCCESS);
    }
    std::printf("%lld derived types, %lld segments compared, %lld bytes located, %lld oracle pack/unpack rounds; "
                "%lld extreme types built, %lld committed\n",
                (long long)g_derived, (long long)g_segments, (long long)g_located, (long long)g_packs,
                (long long)g_extreme_built, (long long)g_extreme_committed);
    std::printf("host sanitize ok\n");
    return 0;
}
