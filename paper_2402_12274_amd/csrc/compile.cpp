// compile.cpp -- commit: compile a type tree into its layout program, lower
// it to the device descriptor, and answer segment queries on the host.
//
// Design (Derived Datatypes, opening paragraphs: a regular layout such as a
// face of a 3-D array is a nested strided vector of constant description
// size; listing its segments would cost O(segments)).  The compiler keeps
// every regular level as a loop (count, byte stride) and only irregular
// levels (indexed, hindexed, struct with unlike members) as a table of
// groups.  Normalisation folds a loop whose stride equals its single run's
// length into the run, merges loops whose strides nest exactly, unrolls tiny
// inner loops into the leaf run list and merges touching leaf runs, so the
// program is as shallow as the layout allows.
//
// Segment queries (Derived Datatypes, Extension): a segment is a maximal run
// that is contiguous in memory and consecutive in map order.  When the
// compiled runs can never touch their successor ("merge-free", the normal
// case), run number k is segment number k and both queries are answered by
// position arithmetic; otherwise a merged segment table is built once.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "core.h"

namespace mdt {

namespace {

bool add_ok(int64_t a, int64_t b, int64_t *r) { return !__builtin_add_overflow(a, b, r); }
bool mul_ok(int64_t a, int64_t b, int64_t *r) { return !__builtin_mul_overflow(a, b, r); }

struct CompileError {
    int code;
};

LayoutP empty_layout()
{
    static LayoutP e = std::make_shared<Layout>();
    return e;
}

int64_t leaf_bytes(const Shape &S)
{
    int64_t u = 0;
    for (const Run &r : S.leaf) u += r.len;
    return u;
}

// packed bytes of one iteration of loop l (l == loops.size(): the leaf)
int64_t span_at(const Shape &S, size_t l)
{
    int64_t s = leaf_bytes(S);
    for (size_t m = l + 1; m < S.loops.size(); m++) s *= S.loops[m].cnt;
    return s;
}

// runs of one iteration of loop l
int64_t runs_at(const Shape &S, size_t l)
{
    int64_t s = (int64_t)S.leaf.size();
    for (size_t m = l + 1; m < S.loops.size(); m++) s *= S.loops[m].cnt;
    return s;
}

int64_t loop0_count(const Shape &S, int64_t glen)
{
    return S.implicit0 ? glen / span_at(S, 0) : S.loops[0].cnt;
}

int64_t group_runs(const Shape &S, int64_t glen)
{
    if (S.varlen) return 1;
    if (S.loops.empty()) return (int64_t)S.leaf.size();
    return loop0_count(S, glen) * runs_at(S, 0);
}

void merge_leaf(std::vector<Run> &leaf)
{
    std::vector<Run> out;
    out.reserve(leaf.size());
    for (const Run &r : leaf) {
        if (r.len == 0) continue;
        if (!out.empty() && out.back().off + out.back().len == r.off) out.back().len += r.len;
        else out.push_back(r);
    }
    leaf.swap(out);
}

constexpr size_t UNROLL_MAX = 8;    // unroll an inner loop into the leaf up to this many runs
constexpr int64_t COLLAPSE_MAX = 64;  // fold a small group list into one leaf list

void normalize(Shape &S)
{
    if (S.varlen) return;
    merge_leaf(S.leaf);
    bool changed = true;
    while (changed) {
        changed = false;
        // drop single-iteration loops (the implicit one keeps its place)
        for (size_t l = 0; l < S.loops.size(); l++) {
            if (S.loops[l].cnt == 1 && !(S.implicit0 && l == 0)) {
                S.loops.erase(S.loops.begin() + l);
                changed = true;
                break;
            }
        }
        if (changed) continue;
        // fold the innermost loop into a single leaf run of matching length
        if (S.leaf.size() == 1 && !S.loops.empty() && S.loops.back().stride == S.leaf[0].len) {
            if (S.implicit0 && S.loops.size() == 1) {
                S.varlen = true;
                S.implicit0 = false;
                S.loops.clear();
                return;
            }
            int64_t len;
            if (mul_ok(S.leaf[0].len, S.loops.back().cnt, &len)) {
                S.leaf[0].len = len;
                S.loops.pop_back();
                changed = true;
                continue;
            }
        }
        // merge loops whose strides nest exactly
        for (size_t l = 0; l + 1 < S.loops.size(); l++) {
            int64_t v, c;
            if (mul_ok(S.loops[l + 1].cnt, S.loops[l + 1].stride, &v) && v == S.loops[l].stride &&
                mul_ok(S.loops[l].cnt, S.loops[l + 1].cnt, &c)) {
                S.loops[l].cnt = (S.implicit0 && l == 0) ? 0 : c;
                S.loops[l].stride = S.loops[l + 1].stride;
                S.loops.erase(S.loops.begin() + l + 1);
                changed = true;
                break;
            }
        }
        if (changed) continue;
        // unroll a tiny innermost loop into the leaf list
        if (!S.loops.empty() && !(S.implicit0 && S.loops.size() == 1)) {
            const Loop lp = S.loops.back();
            if ((size_t)lp.cnt * S.leaf.size() <= UNROLL_MAX) {
                std::vector<Run> nl;
                for (int64_t i = 0; i < lp.cnt; i++)
                    for (const Run &r : S.leaf) {
                        int64_t v, o;
                        if (!mul_ok(i, lp.stride, &v) || !add_ok(r.off, v, &o)) throw CompileError{MDT_ERR_ARG};
                        nl.push_back({o, r.len});
                    }
                merge_leaf(nl);
                S.leaf.swap(nl);
                S.loops.pop_back();
                changed = true;
                continue;
            }
        }
    }
}

int32_t shape_index(std::vector<Shape> &shapes, const Shape &s)
{
    size_t lim = std::min<size_t>(shapes.size(), 256);
    for (size_t i = 0; i < lim; i++)
        if (shapes[i] == s) return (int32_t)i;
    shapes.push_back(s);
    return (int32_t)shapes.size() - 1;
}

void check_groups(size_t n)
{
    if ((int64_t)n > MAX_GROUPS) throw CompileError{MDT_ERR_NO_MEM};
}

// Append the explicit groups of L (outer loops expanded) shifted by base.
void expand_into(const Layout &L, int64_t base, Layout &R)
{
    std::vector<int32_t> map(L.shapes.size());
    for (size_t s = 0; s < L.shapes.size(); s++) map[s] = shape_index(R.shapes, L.shapes[s]);
    size_t no = L.outer.size();
    std::vector<int64_t> idx(no, 0);
    int64_t total = 1;
    for (const Loop &lp : L.outer) total *= lp.cnt;
    check_groups(R.groups.size() + (size_t)total * L.groups.size());
    for (int64_t it = 0; it < total; it++) {
        int64_t addr = base;
        for (size_t l = 0; l < no; l++) addr += idx[l] * L.outer[l].stride;
        for (const Group &g : L.groups) R.groups.push_back({addr + g.disp, g.len, map[g.shape]});
        for (size_t l = no; l-- > 0;) {
            if (++idx[l] < L.outer[l].cnt) break;
            idx[l] = 0;
        }
    }
}

// A single-group layout with a fixed-count shape.
Layout fixed_single(const Layout &L)
{
    Layout R;
    R.size = L.size;
    const Group &g = L.groups[0];
    Shape S = L.shapes[g.shape];
    if (S.varlen) {
        S.varlen = false;
        S.leaf = {{0, g.len}};
    } else if (S.implicit0) {
        S.loops[0].cnt = g.len / span_at(S, 0);
        S.implicit0 = false;
    }
    normalize(S);
    R.shapes.push_back(S);
    R.groups.push_back({g.disp, g.len, 0});
    return R;
}

// Enumerate the runs of one group: f(addr, len) in map order.
template <class F>
void for_each_run(const Shape &S, int64_t disp, int64_t glen, F &&f)
{
    if (S.varlen) {
        f(disp, glen);
        return;
    }
    size_t nl = S.loops.size();
    std::vector<int64_t> cnt(nl), idx(nl, 0);
    for (size_t l = 0; l < nl; l++) cnt[l] = (l == 0 && S.implicit0) ? loop0_count(S, glen) : S.loops[l].cnt;
    for (;;) {
        int64_t a = disp;
        for (size_t l = 0; l < nl; l++) a += idx[l] * S.loops[l].stride;
        for (const Run &r : S.leaf) f(a + r.off, r.len);
        size_t l = nl;
        while (l-- > 0) {
            if (++idx[l] < cnt[l]) break;
            idx[l] = 0;
        }
        if (l == (size_t)-1) break;
    }
}

// Fold a short group list (no outer loops) into one group with a leaf list.
bool collapse(Layout &L)
{
    if (!L.outer.empty() || L.groups.size() <= 1) return false;
    int64_t runs = 0;
    for (const Group &g : L.groups) {
        runs += group_runs(L.shapes[g.shape], g.len);
        if (runs > COLLAPSE_MAX) return false;
    }
    Shape S;
    for (const Group &g : L.groups)
        for_each_run(L.shapes[g.shape], g.disp, g.len, [&](int64_t a, int64_t n) { S.leaf.push_back({a, n}); });
    normalize(S);
    Layout R;
    R.size = L.size;
    R.shapes.push_back(S);
    R.groups.push_back({0, L.size, 0});
    L = std::move(R);
    return true;
}

LayoutP wrap_loop(const LayoutP &L, int64_t cnt, int64_t stride)
{
    if (cnt == 0 || L->size == 0) return empty_layout();
    if (cnt == 1) return L;
    auto R = std::make_shared<Layout>(*L);
    int64_t nsize;
    if (!mul_ok(R->size, cnt, &nsize)) throw CompileError{MDT_ERR_ARG};
    collapse(*R);
    if (R->outer.empty() && R->groups.size() == 1) {
        Layout F = fixed_single(*R);
        F.shapes[0].loops.insert(F.shapes[0].loops.begin(), Loop{cnt, stride});
        normalize(F.shapes[0]);
        F.size = nsize;
        F.groups[0].len = nsize;
        *R = std::move(F);
    } else {
        R->outer.insert(R->outer.begin(), Loop{cnt, stride});
        R->size = nsize;
    }
    return R;
}

LayoutP shifted(const LayoutP &L, int64_t d)
{
    if (d == 0 || L->size == 0) return L;
    auto R = std::make_shared<Layout>(*L);
    for (Group &g : R->groups) g.disp += d;
    return R;
}

// Blocks of copies of child layout CL (extent E): block i has bl[i] copies
// starting at byte shift[i].  Appends to R.
void add_blocks(Layout &R, const LayoutP &CL, int64_t E, const int64_t *shift, const int64_t *bl, int64_t n)
{
    if (CL->size == 0) return;
    if (CL->outer.empty() && CL->groups.size() == 1) {
        Layout F = fixed_single(*CL);
        bool all1 = true;
        for (int64_t i = 0; i < n; i++)
            if (bl[i] != 1 && bl[i] != 0) all1 = false;
        Shape S = F.shapes[0];
        if (!all1) {
            S.loops.insert(S.loops.begin(), Loop{0, E});
            S.implicit0 = true;
            normalize(S);
        }
        int64_t off0 = 0;
        if (S.varlen) {
            off0 = S.leaf.empty() ? 0 : S.leaf[0].off;
            S.leaf.clear();
        }
        int32_t si = shape_index(R.shapes, S);
        int64_t d0 = F.groups[0].disp + off0;
        size_t first = R.groups.size();
        check_groups(first + (size_t)n);
        for (int64_t i = 0; i < n; i++) {
            if (bl[i] == 0) continue;
            int64_t len;
            if (!mul_ok(bl[i], CL->size, &len)) throw CompileError{MDT_ERR_ARG};
            Group g{shift[i] + d0, len, si};
            // touching single-run groups are one run
            if (S.varlen && R.groups.size() > first && R.groups.back().shape == si &&
                R.groups.back().disp + R.groups.back().len == g.disp)
                R.groups.back().len += len;
            else
                R.groups.push_back(g);
        }
    } else {
        for (int64_t i = 0; i < n; i++)
            for (int64_t j = 0; j < bl[i]; j++) expand_into(*CL, shift[i] + j * E, R);
    }
}

LayoutP compile_node(TypeNode *t);

LayoutP child_layout(TypeNode *c) { return compile_node(c); }

LayoutP build(TypeNode *t)
{
    // a type with no data has the empty layout, whatever its parts: their
    // displacements need not even be representable (e.g. copies of a huge
    // extent inside a zero-count vector)
    if (t->size == 0) return empty_layout();
    switch (t->kind) {
    case K_BASIC: {
        auto R = std::make_shared<Layout>();
        Shape S;
        S.leaf.push_back({0, t->size});
        R->shapes.push_back(S);
        R->groups.push_back({0, t->size, 0});
        R->size = t->size;
        return R;
    }
    case K_CONTIG: {
        TypeNode *c = t->kids[0];
        return wrap_loop(child_layout(c), t->n, c->extent());
    }
    case K_VECTOR:
    case K_HVECTOR: {
        TypeNode *c = t->kids[0];
        int64_t E = c->extent();
        int64_t st = t->stride;
        if (t->kind == K_VECTOR && !mul_ok(st, E, &st)) {
            if (t->n > 1) throw CompileError{MDT_ERR_ARG};
            st = 0;
        }
        return wrap_loop(wrap_loop(child_layout(c), t->bl, E), t->n, st);
    }
    case K_HINDEXED: {
        TypeNode *c = t->kids[0];
        auto R = std::make_shared<Layout>();
        add_blocks(*R, child_layout(c), c->extent(), t->disps.data(), t->bls.data(), t->n);
        R->size = t->size;
        if (R->groups.empty()) return empty_layout();
        collapse(*R);
        return R;
    }
    case K_STRUCT: {
        auto R = std::make_shared<Layout>();
        for (int64_t i = 0; i < t->n; i++) {
            TypeNode *c = t->kids[i];
            add_blocks(*R, child_layout(c), c->extent(), &t->disps[i], &t->bls[i], 1);
        }
        R->size = t->size;
        if (R->groups.empty()) return empty_layout();
        collapse(*R);
        return R;
    }
    case K_SUBARRAY: {
        TypeNode *c = t->kids[0];
        int64_t E = c->extent();
        for (int k = 0; k < t->nd; k++)
            if (t->subs[k] == 0) return empty_layout();
        std::vector<int64_t> mult(t->nd);
        int64_t m = 1;
        for (int i = 0; i < t->nd; i++) {
            int k = t->order == MDT_ORDER_C ? t->nd - 1 - i : i;
            mult[k] = m;
            m *= t->sizes[k];
        }
        LayoutP L = child_layout(c);
        int64_t start = 0;
        for (int i = 0; i < t->nd; i++) {
            int k = t->order == MDT_ORDER_C ? t->nd - 1 - i : i;  // innermost first
            L = wrap_loop(L, t->subs[k], mult[k] * E);
            start += t->starts[k] * mult[k] * E;
        }
        return shifted(L, start);
    }
    case K_RESIZED:
    case K_DUP:
        return child_layout(t->kids[0]);
    }
    return empty_layout();
}

LayoutP compile_node(TypeNode *t)
{
    std::lock_guard<std::mutex> g(t->mu);
    if (!t->layout) t->layout = build(t);
    return t->layout;
}

// ---- final form: fit the depth limits ----------------------------------

Layout finalize(const LayoutP &L0)
{
    Layout L = *L0;
    if (L.size == 0 || L.groups.empty()) return Layout{};
    if (L.groups.size() == 1 && L.outer.empty()) L = fixed_single(L);
    // a single group with too many loops: hoist outer loops out of its shape
    if (L.groups.size() == 1 && L.shapes[0].loops.size() > (size_t)MAXI) {
        Shape &S = L.shapes[0];
        while (S.loops.size() > (size_t)MAXI) {
            L.outer.push_back(S.loops.front());
            S.loops.erase(S.loops.begin());
        }
        // the group now holds one iteration of the hoisted loops
        int64_t per = leaf_bytes(S);
        for (const Loop &lp : S.loops) per *= lp.cnt;
        L.groups[0].len = per;
    }
    // expand shapes with too many loops (loop 0 into groups)
    for (bool again = true; again;) {
        again = false;
        for (size_t s = 0; s < L.shapes.size(); s++) {
            if (L.shapes[s].loops.size() <= (size_t)MAXI) continue;
            Shape S = L.shapes[s];
            Shape T = S;
            T.loops.erase(T.loops.begin());
            T.implicit0 = false;
            normalize(T);
            int32_t ti = shape_index(L.shapes, T);
            std::vector<Group> ng;
            for (const Group &g : L.groups) {
                if (g.shape != (int32_t)s) {
                    ng.push_back(g);
                    continue;
                }
                int64_t c0 = loop0_count(S, g.len), sub = g.len / c0;
                check_groups(ng.size() + (size_t)c0);
                for (int64_t i = 0; i < c0; i++) ng.push_back({g.disp + i * S.loops[0].stride, sub, ti});
            }
            L.groups.swap(ng);
            again = true;
            break;
        }
    }
    // too many outer loops: expand the innermost into the group list
    while (L.outer.size() > (size_t)MAXO) {
        Loop lp = L.outer.back();
        L.outer.pop_back();
        std::vector<Group> ng;
        check_groups((size_t)lp.cnt * L.groups.size());
        for (int64_t i = 0; i < lp.cnt; i++)
            for (const Group &g : L.groups) ng.push_back({g.disp + i * lp.stride, g.len, g.shape});
        L.groups.swap(ng);
    }
    // drop unused shapes
    std::vector<int32_t> used(L.shapes.size(), -1);
    std::vector<Shape> ns;
    for (Group &g : L.groups) {
        if (used[g.shape] < 0) {
            used[g.shape] = (int32_t)ns.size();
            ns.push_back(L.shapes[g.shape]);
        }
        g.shape = used[g.shape];
    }
    L.shapes.swap(ns);
    return L;
}

// ---- lowering --------------------------------------------------------------

void lower_shape(const Shape &S, DevShape &D, Compiled &C)
{
    std::memset(&D, 0, sizeof D);
    D.nloops = (int32_t)S.loops.size();
    D.varlen = S.varlen;
    D.implicit0 = S.implicit0;
    D.nleaf = S.varlen ? 0 : (int32_t)S.leaf.size();
    D.unit = leaf_bytes(S);
    for (size_t l = 0; l < S.loops.size(); l++) {
        D.span[l] = span_at(S, l);
        D.stride[l] = S.loops[l].stride;
        D.cnt[l] = S.loops[l].cnt;
        D.rpi[l] = runs_at(S, l);
        D.dspan[l] = make_magic((uint64_t)D.span[l]);
        D.drpi[l] = make_magic((uint64_t)D.rpi[l]);
    }
    // 32-bit positions inside a group: every span and the group itself < 2^31
    // (the group size is checked by the caller for fixed shapes)
    bool small = !S.varlen && !S.implicit0;
    for (size_t l = 0; l < S.loops.size(); l++) small = small && D.span[l] < ((int64_t)1 << 30);
    if (small) {
        for (size_t l = 0; l < S.loops.size(); l++) D.dspan32[l] = make_magic32((uint32_t)D.span[l]);
    }
    D.small32 = small;
    int64_t pre = 0;
    if (D.nleaf <= LEAFI) {
        for (int j = 0; j < D.nleaf; j++) {
            D.loff[j] = S.leaf[j].off;
            D.llen[j] = S.leaf[j].len;
            D.lpre[j] = pre;
            pre += S.leaf[j].len;
        }
        D.lpre[D.nleaf] = pre;
    } else {
        C.leaf_store.emplace_back();
        std::vector<int64_t> &v = C.leaf_store.back();
        size_t n = S.leaf.size();
        v.resize(3 * n + 1);
        for (size_t j = 0; j < n; j++) {
            v[j] = S.leaf[j].off;
            v[n + j] = S.leaf[j].len;
            v[2 * n + j] = pre;
            pre += S.leaf[j].len;
        }
        v[3 * n] = pre;
        // pointers are set by the caller once leaf_store stops growing
    }
}

void set_leaf_ptrs(Compiled &C)
{
    size_t k = 0;
    for (DevShape &D : C.shapes) {
        if (D.nleaf > LEAFI) {
            std::vector<int64_t> &v = C.leaf_store[k++];
            size_t n = (size_t)D.nleaf;
            D.loff_p = v.data();
            D.llen_p = v.data() + n;
            D.lpre_p = v.data() + 2 * n;
        }
    }
}

// last byte end of one group relative to its displacement (runs in map order)
int64_t group_last_end(const Shape &S, int64_t glen)
{
    if (S.varlen) return glen;
    int64_t a = 0;
    for (size_t l = 0; l < S.loops.size(); l++) {
        int64_t c = (l == 0 && S.implicit0) ? loop0_count(S, glen) : S.loops[l].cnt;
        a += (c - 1) * S.loops[l].stride;
    }
    return a + S.leaf.back().off + S.leaf.back().len;
}

int64_t group_first_start(const Shape &S) { return S.varlen ? 0 : S.leaf.front().off; }

// Can a run touch the next one in map order (which would merge them)?
bool compute_merge_free(const Layout &L)
{
    for (const Shape &S : L.shapes) {
        if (S.varlen) continue;
        for (size_t l = 0; l < S.loops.size(); l++) {
            int64_t last = 0;
            for (size_t m = l + 1; m < S.loops.size(); m++) last += (S.loops[m].cnt - 1) * S.loops[m].stride;
            last += S.leaf.back().off + S.leaf.back().len;
            if (S.loops[l].stride + S.leaf.front().off == last) return false;
        }
    }
    for (size_t g = 0; g + 1 < L.groups.size(); g++) {
        const Group &a = L.groups[g], &b = L.groups[g + 1];
        if (a.disp + group_last_end(L.shapes[a.shape], a.len) == b.disp + group_first_start(L.shapes[b.shape]))
            return false;
    }
    if (!L.outer.empty()) {
        const Group &f = L.groups.front(), &b = L.groups.back();
        int64_t first = f.disp + group_first_start(L.shapes[f.shape]);
        int64_t lastg = b.disp + group_last_end(L.shapes[b.shape], b.len);
        for (size_t l = 0; l < L.outer.size(); l++) {
            int64_t last = lastg;
            for (size_t m = l + 1; m < L.outer.size(); m++) last += (L.outer[m].cnt - 1) * L.outer[m].stride;
            if (L.outer[l].stride + first == last) return false;
        }
    }
    return true;
}

// Structural proof that one element's runs are pairwise disjoint.
struct Span {
    int64_t lo, hi;
    bool ok;
};

Span shape_span(const Shape &S, int64_t glen)
{
    if (S.varlen) return {0, glen, true};
    std::vector<Run> lv = S.leaf;
    std::sort(lv.begin(), lv.end(), [](const Run &a, const Run &b) { return a.off < b.off; });
    bool ok = true;
    for (size_t j = 0; j + 1 < lv.size(); j++)
        if (lv[j].off + lv[j].len > lv[j + 1].off) ok = false;
    int64_t lo = lv.front().off, hi = lv.back().off + lv.back().len;
    for (const Run &r : lv) hi = std::max(hi, r.off + r.len);
    for (size_t l = S.loops.size(); l-- > 0;) {
        int64_t c = (l == 0 && S.implicit0) ? loop0_count(S, glen) : S.loops[l].cnt;
        int64_t st = S.loops[l].stride;
        if (c > 1 && (st < 0 ? -st : st) < hi - lo) ok = false;
        int64_t v = (c - 1) * st;
        lo += std::min<int64_t>(0, v);
        hi += std::max<int64_t>(0, v);
    }
    return {lo, hi, ok};
}

bool compute_self_disjoint(const Layout &L)
{
    if (L.groups.empty()) return true;
    std::vector<std::pair<int64_t, int64_t>> iv;
    iv.reserve(L.groups.size());
    for (const Group &g : L.groups) {
        Span s = shape_span(L.shapes[g.shape], g.len);
        if (!s.ok) return false;
        iv.push_back({g.disp + s.lo, g.disp + s.hi});
    }
    std::sort(iv.begin(), iv.end());
    int64_t lo = iv.front().first, hi = iv.front().second;
    for (size_t i = 1; i < iv.size(); i++) {
        if (iv[i].first < hi) return false;
        hi = std::max(hi, iv[i].second);
    }
    for (size_t l = L.outer.size(); l-- > 0;) {
        int64_t c = L.outer[l].cnt, st = L.outer[l].stride;
        if (c > 1 && (st < 0 ? -st : st) < hi - lo) return false;
        int64_t v = (c - 1) * st;
        lo += std::min<int64_t>(0, v);
        hi += std::max<int64_t>(0, v);
    }
    return true;
}

void lower(TypeNode *t, const Layout &L, Compiled &C)
{
    DevLayout &D = C.host;
    std::memset(&D, 0, sizeof D);
    D.size = L.size;
    D.extent = t->extent();
    D.dsize = make_magic((uint64_t)std::max<int64_t>(L.size, 1));
    C.true_lb = t->tlb;
    C.true_ub = t->tub;
    C.extent = t->extent();
    if (L.size == 0) {
        D.kind = KIND_EMPTY;
        C.nruns = 0;
        return;
    }
    const size_t G = L.groups.size();
    C.shapes.resize(L.shapes.size());
    for (size_t s = 0; s < L.shapes.size(); s++) lower_shape(L.shapes[s], C.shapes[s], C);
    set_leaf_ptrs(C);
    D.nshapes = (int32_t)L.shapes.size();
    // a fixed shape's group holds the whole element: 32-bit positions need size < 2^31
    for (size_t s = 0; s < C.shapes.size(); s++)
        if (L.size >= ((int64_t)1 << 30)) C.shapes[s].small32 = 0;
    D.shape0 = C.shapes[0];
    D.G = (int64_t)G;
    D.nouter = (int32_t)L.outer.size();
    if (G == 1 && L.outer.empty()) {
        const Shape &S = L.shapes[0];
        D.gdisp0 = L.groups[0].disp;
        bool contig = S.loops.empty() && S.leaf.size() == 1 && D.extent == L.size;
        D.kind = contig ? KIND_CONTIG : KIND_SINGLE;
        if (contig) D.gdisp0 += S.leaf[0].off;
        D.gsize = L.size;
        D.gruns = S.loops.empty() ? (int64_t)S.leaf.size() : S.loops[0].cnt * runs_at(S, 0);
        D.nruns = D.gruns;
    } else {
        D.kind = KIND_MULTI;
        C.gdisp.resize(G);
        C.gpre.resize(G + 1);
        C.grpre.resize(G + 1);
        if (L.shapes.size() > 1) C.gshape.resize(G);
        int64_t pre = 0, rpre = 0;
        for (size_t g = 0; g < G; g++) {
            const Group &gr = L.groups[g];
            C.gdisp[g] = gr.disp;
            C.gpre[g] = pre;
            C.grpre[g] = rpre;
            if (!C.gshape.empty()) C.gshape[g] = gr.shape;
            pre += gr.len;
            rpre += group_runs(L.shapes[gr.shape], gr.len);
        }
        C.gpre[G] = pre;
        C.grpre[G] = rpre;
        D.gsize = pre;
        D.gruns = rpre;
        // directory: about two groups per cell
        int64_t avg = std::max<int64_t>(1, pre / (int64_t)G);
        int sh = 4;
        while (sh < 40 && ((int64_t)1 << sh) < 2 * avg) sh++;
        int64_t ndir = (pre + ((int64_t)1 << sh) - 1) >> sh;
        C.gdir.resize((size_t)ndir);
        int64_t g = 0;
        for (int64_t k = 0; k < ndir; k++) {
            int64_t b = k << sh;
            while (C.gpre[g + 1] <= b) g++;
            C.gdir[k] = (int32_t)g;
        }
        D.dir_shift = sh;
        D.ndir = ndir;
        int64_t ospan = pre, orun = rpre;
        for (size_t l = L.outer.size(); l-- > 0;) {
            D.ospan[l] = ospan;
            D.orun[l] = orun;
            D.ostride[l] = L.outer[l].stride;
            D.ocnt[l] = L.outer[l].cnt;
            D.dospan[l] = make_magic((uint64_t)ospan);
            D.dorun[l] = make_magic((uint64_t)orun);
            ospan *= L.outer[l].cnt;
            orun *= L.outer[l].cnt;
        }
        D.nruns = orun;
        D.runs_only = L.outer.empty() && L.shapes.size() == 1 && L.shapes[0].varlen;
        D.gdisp = C.gdisp.data();
        D.gpre = C.gpre.data();
        D.grpre = C.grpre.data();
        D.gshape = C.gshape.empty() ? nullptr : C.gshape.data();
        D.gdir = C.gdir.data();
        D.shapes = C.shapes.data();
    }
    C.nruns = D.nruns;
    C.merge_free = compute_merge_free(L);
    C.self_disjoint = compute_self_disjoint(L);
}

// Record view of a single-group layout: records are the count elements
// (shape without loops) or the iterations of the shape's only loop.
void lower_records(const Layout &L, Compiled &C)
{
    DevLayout &D = C.host;
    DevRecords &R = D.rec;
    std::memset(&R, 0, sizeof R);
    if (D.kind != KIND_SINGLE) return;
    const Shape &S = L.shapes[0];
    int64_t X, U = leaf_bytes(S);
    bool count1 = false;
    if (S.loops.empty()) {
        X = D.extent;
    } else if (S.loops.size() == 1) {
        X = S.loops[0].stride;
        int64_t span;
        count1 = !mul_ok(S.loops[0].cnt, S.loops[0].stride, &span) || D.extent != span;
    } else {
        return;
    }
    if (X <= 0 || X > REC_MAX_X || U < 1 || U > REC_MAX_U || X > 4 * U) return;
    // records of long runs move at full speed on the chunk path (one run per
    // 16-byte chunk, whole tiles inside one run); staging them in LDS only
    // shrinks the grid
    if (U >= REC_MIN_RUN * (int64_t)S.leaf.size()) return;
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    for (const Run &r : S.leaf) {
        lo = std::min(lo, r.off);
        hi = std::max(hi, r.off + r.len);
    }
    if (hi - lo > 65535) return;
    // packed -> typed byte table (pack)
    C.rec_ptab.assign((size_t)U, 0);
    int64_t q = 0;
    for (const Run &r : S.leaf)
        for (int64_t i = 0; i < r.len; i++, q++)
            C.rec_ptab[q] = (uint32_t)(r.off + i - lo) | (uint32_t)(r.len - i) << 16;
    // typed -> packed byte table (unpack), when records do not interleave and
    // no byte of a record is covered twice
    bool ok = hi - lo <= X;
    if (ok) {
        C.rec_ttab.assign((size_t)X, 0);
        q = 0;
        for (const Run &r : S.leaf) {
            for (int64_t i = 0; i < r.len; i++) {
                uint32_t &e = C.rec_ttab[r.off + i - lo];
                if (e & 0x80000000u) ok = false;
                e = 0x80000000u | (uint32_t)(q + i) | (uint32_t)std::min<int64_t>(r.len - i, 0x7fff) << 16;
            }
            q += r.len;
        }
    }
    if (!ok) C.rec_ttab.clear();
    // chunk table: the 16 typed offsets of the packed chunk starting at q
    const bool ctab = U <= REC_CTAB_MAX_U;
    C.rec_ctab.clear();
    if (ctab) {
        C.rec_ctab.resize((size_t)U * 16);
        for (int64_t qq = 0; qq < U; qq++)
            for (int64_t j = 0; j < 16; j++) {
                int64_t pos = qq + j, rr = pos / U;
                C.rec_ctab[(size_t)(qq * 16 + j)] = (C.rec_ptab[(size_t)(pos - rr * U)] & 0xffffu) + (uint32_t)(rr * X);
            }
    }
    // dword table: packed offsets and coverage of typed bytes d .. d + 3
    const bool dtab = ok && X >= 4 && X <= REC_DTAB_MAX_X;
    C.rec_dtab.clear();
    if (dtab) {
        C.rec_dtab.assign((size_t)X * 4, 0);
        for (int64_t d = 0; d < X; d++) {
            uint32_t *e = &C.rec_dtab[(size_t)(4 * d)];
            for (int i = 0; i < 4; i++) {
                int64_t t = d + i, rr = t >= X ? 1 : 0;
                uint32_t te = C.rec_ttab[(size_t)(t - rr * X)];
                if (!(te & 0x80000000u)) continue;
                uint32_t pq = (te & 0xffffu) + (uint32_t)(rr * U);
                e[i >> 1] |= pq << (16 * (i & 1));
                e[2] |= 1u << i;
            }
        }
    }
    // LDS for a tile: the table in front, then the typed span (pack) or the
    // packed window (unpack), with slack for rounding out to 16-byte blocks
    static const int tc_max = [] {
        const char *e = getenv("MDT_DENSE_TILE");
        int v = e && *e ? atoi(e) : 1024;
        return v >= 64 && v <= 2048 ? v : 1024;
    }();
    auto a16 = [](int64_t n) { return (n + 15) & ~(int64_t)15; };
    auto need = [&](int c) {
        int64_t nrec = (16 * (int64_t)c + U - 1) / U + 1;
        int64_t span = (nrec - 1) * X + (hi - lo) + 48;
        int64_t np = a16(ctab ? 64 * U : 4 * U) + a16(span) + 16;
        int64_t nu = 0;
        if (ok) nu = dtab ? a16(16 * X) + a16(16 * (int64_t)c + 4 * U + 64) + 16 : a16(4 * X) + a16(16 * (int64_t)c + 48) + 16;
        return std::max(np, nu);
    };
    int tc = tc_max;
    while (tc > 64 && need(tc) > 40 * 1024) tc /= 2;
    if (need(tc) > 40 * 1024) {
        C.rec_ptab.clear();
        C.rec_ttab.clear();
        C.rec_ctab.clear();
        C.rec_dtab.clear();
        return;
    }
    R.on = 1;
    R.U = (int32_t)U;
    R.X = (int32_t)X;
    R.lo = (int32_t)lo;
    R.hi = (int32_t)hi;
    R.unpack_ok = ok;
    R.B0 = L.groups[0].disp;
    R.dU = make_magic((uint64_t)U);
    R.dU32 = make_magic32((uint32_t)U);
    R.dX32 = make_magic32((uint32_t)X);
    R.tile_chunks = tc;
    R.lds_bytes = (int32_t)need(tc);
    R.ptab = C.rec_ptab.data();
    R.ttab = ok ? C.rec_ttab.data() : nullptr;
    R.ctab = ctab ? C.rec_ctab.data() : nullptr;
    R.dtab = dtab ? C.rec_dtab.data() : nullptr;
    C.rec_count1_only = count1;
    R.count1_only = count1;
}

std::shared_ptr<Compiled> make_compiled(TypeNode *t)
{
    LayoutP L0 = compile_node(t);
    auto C = std::make_shared<Compiled>();
    C->layout = std::make_shared<Layout>(finalize(L0));
    lower(t, *C->layout, *C);
    lower_records(*C->layout, *C);
    return C;
}

// run number and run start of byte q (< size) of one element
void run_of_byte(const Compiled &C, int64_t q, int64_t *k, int64_t *start)
{
    const DevLayout &L = C.host;
    int64_t pos = q, r = 0;
    const DevShape *S = &L.shape0;
    int64_t glen = L.size;
    if (L.kind == KIND_CONTIG) {
        *k = 0;
        *start = 0;
        return;
    }
    if (L.kind == KIND_MULTI) {
        for (int l = 0; l < L.nouter; l++) {
            int64_t i = q / L.ospan[l];
            q -= i * L.ospan[l];
            r += i * L.orun[l];
        }
        int64_t g = find_group(L, (uint64_t)q);
        q -= L.gpre[g];
        r += L.grpre[g];
        glen = L.gpre[g + 1] - L.gpre[g];
        S = &L.shapes[L.nshapes == 1 ? 0 : L.gshape[g]];
    }
    (void)glen;
    if (S->varlen) {
        *k = r;
        *start = pos - q;
        return;
    }
    for (int l = 0; l < S->nloops; l++) {
        int64_t i = q / S->span[l];
        q -= i * S->span[l];
        r += i * S->rpi[l];
    }
    int j = 0;
    while (j + 1 < S->nleaf && leaf_at(*S, (uint64_t)(j + 1)).pre <= q) j++;
    *k = r + j;
    *start = pos - (q - leaf_at(*S, (uint64_t)j).pre);
}

}  // namespace

Compiled::~Compiled()
{
    for (auto &d : dev)
        if (d) free_device_tables(d.get());
}

int compile_layout(TypeNode *t, LayoutP *out)
{
    try {
        *out = compile_node(t);
    } catch (const CompileError &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        return MDT_ERR_NO_MEM;
    }
    return MDT_SUCCESS;
}

int commit_type(TypeNode *t)
{
    if (t->committed.load()) return MDT_SUCCESS;
    std::shared_ptr<Compiled> C;
    try {
        C = make_compiled(t);
    } catch (const CompileError &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        return MDT_ERR_NO_MEM;
    }
    {
        std::lock_guard<std::mutex> g(t->mu);
        if (!t->comp) t->comp = C;
        C = t->comp;
    }
    // resident device tables when a device is present (otherwise on first use)
    DeviceTables *d = nullptr;
    int rc = device_tables(C.get(), &d);
    if (rc != MDT_SUCCESS && rc != MDT_ERR_HIP) return rc;
    t->committed.store(true);
    return MDT_SUCCESS;
}

int build_segment_table(Compiled *c)
{
    std::call_once(c->seg_once, [c]() {
        try {
            if (c->nruns > MAX_SEG_TABLE) {
                c->seg_status = MDT_ERR_NO_MEM;
                return;
            }
            int64_t pre = 0;
            for (int64_t k = 0; k < c->nruns; k++) {
                RunInfo r = run_at(c->host, (uint64_t)k);
                if (!c->seg_addr.empty() && c->seg_addr.back() + c->seg_len.back() == r.addr) {
                    c->seg_len.back() += r.len;
                } else {
                    c->seg_addr.push_back(r.addr);
                    c->seg_len.push_back(r.len);
                    c->seg_pre.push_back(pre);
                }
                pre += r.len;
            }
            c->seg_pre.push_back(pre);
        } catch (...) {
            c->seg_status = MDT_ERR_NO_MEM;
        }
    });
    return c->seg_status;
}

int host_iov_len(TypeNode *t, int64_t max_bytes, int64_t *n, int64_t *bytes)
{
    int rc = commit_type(t);
    if (rc) return rc;
    Compiled *C = t->comp.get();
    int64_t nseg;
    if (!C->merge_free) {
        rc = build_segment_table(C);
        if (rc) return rc;
        nseg = (int64_t)C->seg_addr.size();
    } else {
        nseg = C->nruns;
    }
    if (max_bytes == -1 || max_bytes >= t->size) {
        *n = nseg;
        *bytes = t->size;
        return MDT_SUCCESS;
    }
    if (C->merge_free) {
        int64_t k, start;
        run_of_byte(*C, max_bytes, &k, &start);
        *n = k;
        *bytes = start;
    } else {
        // segment containing byte max_bytes: last k with pre[k] <= max
        auto it = std::upper_bound(C->seg_pre.begin(), C->seg_pre.end(), max_bytes);
        int64_t k = (int64_t)(it - C->seg_pre.begin()) - 1;
        *n = k;
        *bytes = C->seg_pre[k];
    }
    return MDT_SUCCESS;
}

int host_iov(TypeNode *t, int64_t off, mdt_iov *iov, int64_t m, int64_t *actual)
{
    int rc = commit_type(t);
    if (rc) return rc;
    Compiled *C = t->comp.get();
    if (!C->merge_free) {
        rc = build_segment_table(C);
        if (rc) return rc;
        int64_t nseg = (int64_t)C->seg_addr.size();
        int64_t end = off >= nseg ? off : std::min(nseg, off + m);
        for (int64_t k = off; k < end; k++) {
            iov[k - off].iov_base = (void *)(intptr_t)C->seg_addr[k];
            iov[k - off].iov_len = C->seg_len[k];
        }
        *actual = end - off;
        return MDT_SUCCESS;
    }
    int64_t nseg = C->nruns;
    int64_t end = off >= nseg ? off : std::min(nseg, off + m);
    for (int64_t k = off; k < end; k++) {
        RunInfo r = run_at(C->host, (uint64_t)k);
        iov[k - off].iov_base = (void *)(intptr_t)r.addr;
        iov[k - off].iov_len = r.len;
    }
    *actual = end - off;
    return MDT_SUCCESS;
}

// ---- segments of count consecutive elements --------------------------
//
// Element r is the element's typemap shifted by r * extent, so the count
// form's segments are the element's segments repeated, except where the
// element's last segment ends exactly where the next element's first one
// starts (first_addr + extent == last_end): those two merge across the
// boundary.  With n element segments that gives 1 + count*(n-1) segments
// (one in all when n = 1), in the order seg 0 of element 0, then for each
// element q its segments 1..n-2 followed by the bridge (its last segment
// merged with element q+1's first; element count-1's last stands alone).

int element_segments(TypeNode *t, SegCount *sc, int64_t count)
{
    int rc = commit_type(t);
    if (rc) return rc;
    Compiled *C = t->comp.get();
    if (!C->merge_free) {
        rc = build_segment_table(C);
        if (rc) return rc;
    }
    if (count < 0) return MDT_ERR_ARG;
    int64_t x;
    if (__builtin_mul_overflow(count, t->size, &x) || __builtin_mul_overflow(count, t->extent(), &x))
        return MDT_ERR_COUNT;
    sc->C = C;
    sc->count = count;
    sc->extent = t->extent();
    sc->size = t->size;
    sc->n = C->merge_free ? C->nruns : (int64_t)C->seg_addr.size();
    sc->merge = false;
    if (sc->n > 0 && count > 1) {
        int64_t a0, l0, al, ll;
        seg_of(*sc, 0, &a0, &l0);
        seg_of(*sc, sc->n - 1, &al, &ll);
        sc->merge = a0 + sc->extent == al + ll;
    }
    if (count == 0 || sc->n == 0) sc->total = 0;
    else if (!sc->merge) {
        if (__builtin_mul_overflow(count, sc->n, &sc->total)) return MDT_ERR_COUNT;
    } else sc->total = sc->n == 1 ? 1 : 1 + count * (sc->n - 1);
    return MDT_SUCCESS;
}

// segment j (< n) of one element
void seg_of(const SegCount &sc, int64_t j, int64_t *addr, int64_t *len)
{
    if (sc.C->merge_free) {
        RunInfo r = run_at(sc.C->host, (uint64_t)j);
        *addr = r.addr;
        *len = r.len;
    } else {
        *addr = sc.C->seg_addr[(size_t)j];
        *len = sc.C->seg_len[(size_t)j];
    }
}

// segment g (< total) of the count form
void seg_count_at(const SegCount &sc, int64_t g, int64_t *addr, int64_t *len)
{
    if (!sc.merge) {
        const int64_t q = g / sc.n, j = g % sc.n;
        seg_of(sc, j, addr, len);
        *addr += q * sc.extent;
        return;
    }
    if (sc.n == 1) {
        seg_of(sc, 0, addr, len);
        *len *= sc.count;
        return;
    }
    if (g == 0) {
        seg_of(sc, 0, addr, len);
        return;
    }
    const int64_t q = (g - 1) / (sc.n - 1), j = (g - 1) % (sc.n - 1) + 1;
    seg_of(sc, j, addr, len);
    *addr += q * sc.extent;
    if (j == sc.n - 1 && q < sc.count - 1) {
        int64_t a0, l0;
        seg_of(sc, 0, &a0, &l0);
        *len += l0;
    }
}

int host_iov_len_count(TypeNode *t, int64_t count, int64_t max_bytes, int64_t *n, int64_t *bytes)
{
    SegCount sc{};
    int rc = element_segments(t, &sc, count);
    if (rc) return rc;
    const int64_t all = count * t->size;
    if (max_bytes == -1 || max_bytes >= all) {
        *n = sc.total;
        *bytes = all;
        return MDT_SUCCESS;
    }
    // max_bytes < all, so the element size is positive: byte max_bytes lies
    // in element r at rem, inside element segment j (P_j <= rem < P_{j+1})
    int64_t r = max_bytes / t->size, rem = max_bytes - r * t->size, j, pj;
    if (sc.C->merge_free) {
        run_of_byte(*sc.C, rem, &j, &pj);
    } else {
        auto it = std::upper_bound(sc.C->seg_pre.begin(), sc.C->seg_pre.end(), rem);
        j = (int64_t)(it - sc.C->seg_pre.begin()) - 1;
        pj = sc.C->seg_pre[(size_t)j];
    }
    if (!sc.merge) {
        *n = r * sc.n + j;
        *bytes = r * t->size + pj;
        return MDT_SUCCESS;
    }
    if (sc.n == 1 || (r == 0 && j == 0)) {  // inside the first segment
        *n = 0;
        *bytes = 0;
        return MDT_SUCCESS;
    }
    if (j == 0) {  // element r's first bytes belong to the bridge from element r-1
        r -= 1;
        j = sc.n - 1;
        pj = t->size - (sc.C->merge_free ? run_at(sc.C->host, (uint64_t)j).len : sc.C->seg_len[(size_t)j]);
    }
    *n = 1 + r * (sc.n - 1) + (j - 1);
    *bytes = r * t->size + pj;
    return MDT_SUCCESS;
}

int host_iov_count(TypeNode *t, int64_t count, int64_t off, mdt_iov *iov, int64_t m, int64_t *actual)
{
    SegCount sc{};
    int rc = element_segments(t, &sc, count);
    if (rc) return rc;
    const int64_t end = off >= sc.total ? off : std::min(sc.total, off + m);
    for (int64_t g = off; g < end; g++) {
        int64_t a, l;
        seg_count_at(sc, g, &a, &l);
        iov[g - off].iov_base = (void *)(intptr_t)a;
        iov[g - off].iov_len = l;
    }
    *actual = end - off;
    return MDT_SUCCESS;
}

int check_unpack_overlap(Compiled *c, int64_t count)
{
    std::lock_guard<std::mutex> g(c->ov_mu);
    if (count <= c->ov_checked_count) return MDT_SUCCESS;
    if (c->nruns == 0) return MDT_SUCCESS;  // no bytes, nothing to overlap (and no loop over count)
    // every element's address must be representable (callers check this too)
    int64_t span, lo, hi;
    if (count > 1 && (__builtin_mul_overflow(count - 1, c->extent, &span) ||
                      __builtin_add_overflow(span, c->true_lb, &lo) || __builtin_add_overflow(span, c->true_ub, &hi)))
        return MDT_ERR_COUNT;
    int64_t te = c->true_ub - c->true_lb;
    int64_t ae = c->extent < 0 ? -c->extent : c->extent;
    if (c->self_disjoint && (count <= 1 || ae >= te)) {
        c->ov_checked_count = INT64_MAX;
        if (count <= 1 && ae < te) c->ov_checked_count = 1;
        return MDT_SUCCESS;
    }
    // exact check: every run of every element, sorted by address
    int64_t total;
    if (__builtin_mul_overflow(count, c->nruns, &total) || total > MAX_OVERLAP_RUNS) return MDT_ERR_NO_MEM;
    std::vector<std::pair<int64_t, int64_t>> runs;
    try {
        runs.reserve((size_t)total);
        for (int64_t r = 0; r < count; r++)
            for (int64_t k = 0; k < c->nruns; k++) {
                RunInfo ri = run_at(c->host, (uint64_t)k);
                runs.push_back({r * c->extent + ri.addr, ri.len});
            }
    } catch (...) {
        return MDT_ERR_NO_MEM;
    }
    std::sort(runs.begin(), runs.end());
    for (size_t i = 0; i + 1 < runs.size(); i++)
        if (runs[i].first + runs[i].second > runs[i + 1].first) return MDT_ERR_OVERLAP;
    c->ov_checked_count = count;
    return MDT_SUCCESS;
}

}  // namespace mdt
