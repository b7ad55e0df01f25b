/*
 * oracle.c -- plain recursive typemap walker (TEST INFRASTRUCTURE ONLY).
 *
 * What it follows:
 *  - Derived Datatypes section, opening paragraphs: a datatype describes a
 *    (possibly nested, offset, overlapping) memory layout; its segments are
 *    what an iovec listing of that layout would contain.
 *  - Derived Datatypes, Extension: MPIX_Type_iov_len (whole segments inside
 *    a byte budget; -1 or more than the type size means all of them) and
 *    MPIX_Type_iov (segments from an index, at most a given number), with
 *    MPIX_Iov = {base, len}.
 *  - Derived Datatypes, Example: the constructors used there (contiguous,
 *    subarray) and the commit/free life cycle.
 *  - The constructors' typemaps themselves follow the MPI standard's
 *    definitions, which the paper relies on without restating them; each
 *    one is written out below as the list of child copies it places, in
 *    emission order.
 *  - General Progress, Background: large messages are moved as pipelined
 *    chunks, hence pack/unpack of a byte range [offset, offset + budget) of
 *    the packed stream.
 *
 * Nothing here is tuned.  Every entry is visited one by one; the only
 * shortcut is that pack/unpack skip a whole child copy whose bytes all lie
 * before the requested range (its packed size is known), which leaves the
 * copied bytes unchanged.
 */
#include "oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef enum {
    K_BASIC,
    K_CONTIG,
    K_VECTOR,
    K_HVECTOR,
    K_INDEXED,
    K_HINDEXED,
    K_STRUCT,
    K_SUBARRAY,
    K_RESIZED,
    K_DUP,
    K_DARRAY
} kind_t;

#define ORC_MAX_DIMS 32

struct orc_type {
    int refs;
    kind_t kind;
    int64_t n;      /* copies / blocks */
    int64_t bl;     /* vector / hvector block length */
    int64_t stride; /* vector: in child extents; hvector: in bytes */
    int64_t *bls;   /* per-block lengths (indexed, hindexed, struct) */
    int64_t *disps; /* per-block displacements (indexed: extents; others: bytes) */
    orc_type **kids;
    orc_type *child;
    int nd, order;
    int64_t *sizes, *subs, *starts;
    int64_t *own, *own_off; /* darray: owned indices of each dimension */
    int64_t rlb, rext;
    /* attributes */
    int64_t size, lb, ub, tlb, tub, align, nent;
    int expl;
};

/* ------------------------------------------------------------------ */
/* checked arithmetic                                                   */

static int add_ok(int64_t a, int64_t b, int64_t *r) { return !__builtin_add_overflow(a, b, r); }
static int mul_ok(int64_t a, int64_t b, int64_t *r) { return !__builtin_mul_overflow(a, b, r); }

static int64_t extent_of(const orc_type *t) { return t->ub - t->lb; }

/* ------------------------------------------------------------------ */
/* copy enumeration: the typemap of every constructor as a list of child
 * copies (shift, child), in emission order.  The callback returns nonzero
 * to stop.  Return: 0 done, 1 stopped, -1 displacement overflow.          */

typedef int (*copy_cb)(void *ctx, int64_t shift, const orc_type *c);

static int for_each_copy(const orc_type *t, copy_cb cb, void *ctx)
{
    int64_t i, j, s, a, b;
    switch (t->kind) {
    case K_BASIC:
        return 0;
    case K_CONTIG: {
        /* contiguous(n, c): copy i at i * extent(c) */
        int64_t E = extent_of(t->child);
        for (i = 0; i < t->n; i++) {
            if (!mul_ok(i, E, &s)) return -1;
            if (cb(ctx, s, t->child)) return 1;
        }
        return 0;
    }
    case K_VECTOR: {
        /* vector(n, bl, stride, c): copy (i, j) at (i*stride + j) * extent(c) */
        int64_t E = extent_of(t->child);
        for (i = 0; i < t->n; i++)
            for (j = 0; j < t->bl; j++) {
                if (!mul_ok(i, t->stride, &a) || !add_ok(a, j, &a) || !mul_ok(a, E, &s)) return -1;
                if (cb(ctx, s, t->child)) return 1;
            }
        return 0;
    }
    case K_HVECTOR: {
        /* hvector(n, bl, stride_bytes, c): copy (i, j) at i*stride + j*extent(c) */
        int64_t E = extent_of(t->child);
        for (i = 0; i < t->n; i++)
            for (j = 0; j < t->bl; j++) {
                if (!mul_ok(i, t->stride, &a) || !mul_ok(j, E, &b) || !add_ok(a, b, &s)) return -1;
                if (cb(ctx, s, t->child)) return 1;
            }
        return 0;
    }
    case K_INDEXED: {
        /* indexed(n, bl[], disp[], c): copy (i, j) at (disp[i] + j) * extent(c) */
        int64_t E = extent_of(t->child);
        for (i = 0; i < t->n; i++)
            for (j = 0; j < t->bls[i]; j++) {
                if (!add_ok(t->disps[i], j, &a) || !mul_ok(a, E, &s)) return -1;
                if (cb(ctx, s, t->child)) return 1;
            }
        return 0;
    }
    case K_HINDEXED: {
        /* hindexed(n, bl[], disp_bytes[], c): copy (i, j) at disp[i] + j*extent(c) */
        int64_t E = extent_of(t->child);
        for (i = 0; i < t->n; i++)
            for (j = 0; j < t->bls[i]; j++) {
                if (!mul_ok(j, E, &b) || !add_ok(t->disps[i], b, &s)) return -1;
                if (cb(ctx, s, t->child)) return 1;
            }
        return 0;
    }
    case K_STRUCT: {
        /* struct(n, bl[], disp_bytes[], c[]): copy (i, j) of c[i] at disp[i] + j*extent(c[i]) */
        for (i = 0; i < t->n; i++) {
            int64_t E = extent_of(t->kids[i]);
            for (j = 0; j < t->bls[i]; j++) {
                if (!mul_ok(j, E, &b) || !add_ok(t->disps[i], b, &s)) return -1;
                if (cb(ctx, s, t->kids[i])) return 1;
            }
        }
        return 0;
    }
    case K_SUBARRAY: {
        /* subarray: every index tuple of the sub-box, the last dimension
         * varying fastest for C order and the first for Fortran order; the
         * copy sits at lin(tuple) * extent(c), lin being the row-major (C)
         * or column-major (Fortran) linear index inside the full array. */
        int nd = t->nd, k;
        int64_t idx[ORC_MAX_DIMS], mult[ORC_MAX_DIMS];
        int64_t E = extent_of(t->child);
        for (k = 0; k < nd; k++) {
            if (t->subs[k] == 0) return 0;
            idx[k] = t->starts[k];
        }
        if (t->order == ORC_ORDER_C) {
            int64_t m = 1;
            for (k = nd - 1; k >= 0; k--) { mult[k] = m; if (!mul_ok(m, t->sizes[k], &m)) m = INT64_MAX; }
        } else {
            int64_t m = 1;
            for (k = 0; k < nd; k++) { mult[k] = m; if (!mul_ok(m, t->sizes[k], &m)) m = INT64_MAX; }
        }
        for (;;) {
            int64_t lin = 0;
            for (k = 0; k < nd; k++) {
                if (!mul_ok(idx[k], mult[k], &a) || !add_ok(lin, a, &lin)) return -1;
            }
            if (!mul_ok(lin, E, &s)) return -1;
            if (cb(ctx, s, t->child)) return 1;
            /* advance the odometer, fastest dimension first */
            if (t->order == ORC_ORDER_C) {
                for (k = nd - 1; k >= 0; k--) {
                    if (++idx[k] < t->starts[k] + t->subs[k]) break;
                    idx[k] = t->starts[k];
                }
            } else {
                for (k = 0; k < nd; k++) {
                    if (++idx[k] < t->starts[k] + t->subs[k]) break;
                    idx[k] = t->starts[k];
                }
                if (k == nd) k = -1;
            }
            if (k < 0) return 0;
        }
    }
    case K_DARRAY: {
        /* distributed array: every tuple of owned indices (each dimension's
         * owned indices in increasing order), the last dimension varying
         * fastest for C order and the first for Fortran order; the copy
         * sits at lin(tuple) * extent(c) over the global array. */
        int nd = t->nd, k;
        int64_t pos[ORC_MAX_DIMS], mult[ORC_MAX_DIMS];
        int64_t E = extent_of(t->child);
        for (k = 0; k < nd; k++) {
            if (t->own_off[k + 1] == t->own_off[k]) return 0;
            pos[k] = 0;
        }
        if (t->order == ORC_ORDER_C) {
            int64_t m = 1;
            for (k = nd - 1; k >= 0; k--) { mult[k] = m; if (!mul_ok(m, t->sizes[k], &m)) m = INT64_MAX; }
        } else {
            int64_t m = 1;
            for (k = 0; k < nd; k++) { mult[k] = m; if (!mul_ok(m, t->sizes[k], &m)) m = INT64_MAX; }
        }
        for (;;) {
            int64_t lin = 0;
            for (k = 0; k < nd; k++) {
                if (!mul_ok(t->own[t->own_off[k] + pos[k]], mult[k], &a) || !add_ok(lin, a, &lin)) return -1;
            }
            if (!mul_ok(lin, E, &s)) return -1;
            if (cb(ctx, s, t->child)) return 1;
            if (t->order == ORC_ORDER_C) {
                for (k = nd - 1; k >= 0; k--) {
                    if (++pos[k] < t->own_off[k + 1] - t->own_off[k]) break;
                    pos[k] = 0;
                }
            } else {
                for (k = 0; k < nd; k++) {
                    if (++pos[k] < t->own_off[k + 1] - t->own_off[k]) break;
                    pos[k] = 0;
                }
                if (k == nd) k = -1;
            }
            if (k < 0) return 0;
        }
    }
    case K_RESIZED:
    case K_DUP:
        /* the typemap of the child, unchanged */
        return cb(ctx, 0, t->child) ? 1 : 0;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* attributes                                                           */

typedef struct {
    int placed, data, ovf;
    int64_t lb, ub, tlb, tub, size, align, nent;
    int expl;
} attr_acc;

static int attr_cb(void *ctx, int64_t shift, const orc_type *c)
{
    attr_acc *A = (attr_acc *)ctx;
    int64_t v;
    /* lb / ub: over every placed copy, of shift + lb(c) and shift + ub(c) */
    if (!add_ok(shift, c->lb, &v)) { A->ovf = 1; return 1; }
    if (!A->placed || v < A->lb) A->lb = v;
    if (!add_ok(shift, c->ub, &v)) { A->ovf = 1; return 1; }
    if (!A->placed || v > A->ub) A->ub = v;
    A->placed = 1;
    /* true bounds: over the copies that carry bytes */
    if (c->size > 0) {
        if (!add_ok(shift, c->tlb, &v)) { A->ovf = 1; return 1; }
        if (!A->data || v < A->tlb) A->tlb = v;
        if (!add_ok(shift, c->tub, &v)) { A->ovf = 1; return 1; }
        if (!A->data || v > A->tub) A->tub = v;
        A->data = 1;
    }
    if (!add_ok(A->size, c->size, &A->size)) { A->ovf = 1; return 1; }
    if (!add_ok(A->nent, c->nent, &A->nent)) { A->ovf = 1; return 1; }
    if (c->align > A->align) A->align = c->align;
    A->expl |= c->expl;
    return 0;
}

/* Fill in the attributes of a freshly built non-basic node.  Returns
 * ORC_OK or ORC_ERR_ARG on overflow. */
static int compute_attrs(orc_type *t)
{
    attr_acc A;
    memset(&A, 0, sizeof A);
    A.align = 1;
    if (for_each_copy(t, attr_cb, &A) < 0 || A.ovf) return ORC_ERR_ARG;
    t->size = A.size;
    t->nent = A.nent;
    t->align = A.align;
    t->expl = A.expl;
    t->lb = A.placed ? A.lb : 0;
    t->ub = A.placed ? A.ub : 0;
    t->tlb = A.data ? A.tlb : 0;
    t->tub = A.data ? A.tub : 0;
    switch (t->kind) {
    case K_STRUCT:
        /* natural alignment padding: the extent of a struct is rounded up to
         * a multiple of its largest member alignment, unless a member
         * carries explicit bounds (a resized or subarray type). */
        if (!A.expl && A.placed) {
            int64_t ext = t->ub - t->lb;
            if (ext > 0 && ext % A.align != 0) {
                int64_t pad = A.align - ext % A.align;
                if (!add_ok(t->ub, pad, &t->ub)) return ORC_ERR_ARG;
            }
        }
        break;
    case K_SUBARRAY:
    case K_DARRAY: {
        /* bounds are those of the whole array: [0, prod(sizes) * extent) */
        int64_t m = 1;
        int k;
        for (k = 0; k < t->nd; k++)
            if (!mul_ok(m, t->sizes[k], &m)) return ORC_ERR_ARG;
        if (!mul_ok(m, extent_of(t->child), &m)) return ORC_ERR_ARG;
        t->lb = 0;
        t->ub = m;
        t->expl = 1;
        break;
    }
    case K_RESIZED:
        t->lb = t->rlb;
        if (!add_ok(t->rlb, t->rext, &t->ub)) return ORC_ERR_ARG;
        t->expl = 1;
        break;
    default:
        break;
    }
    {
        int64_t e;
        if (__builtin_sub_overflow(t->ub, t->lb, &e)) return ORC_ERR_ARG;
        if (__builtin_sub_overflow(t->tub, t->tlb, &e)) return ORC_ERR_ARG;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* construction                                                         */

static orc_type *new_node(kind_t k)
{
    orc_type *t = (orc_type *)calloc(1, sizeof *t);
    if (t) {
        t->refs = 1;
        t->kind = k;
    }
    return t;
}

static void retain(orc_type *t) { t->refs++; }

void orc_release(orc_type *t)
{
    int64_t i;
    if (!t || --t->refs > 0) return;
    if (t->child) orc_release(t->child);
    if (t->kids) {
        for (i = 0; i < t->n; i++) orc_release(t->kids[i]);
        free(t->kids);
    }
    free(t->bls);
    free(t->disps);
    free(t->sizes);
    free(t->subs);
    free(t->starts);
    free(t->own);
    free(t->own_off);
    free(t);
}

static orc_type *finish(orc_type *t, int *err)
{
    int rc = compute_attrs(t);
    if (rc != ORC_OK) {
        orc_release(t);
        if (err) *err = rc;
        return NULL;
    }
    if (err) *err = ORC_OK;
    return t;
}

static orc_type *fail(int *err, int code)
{
    if (err) *err = code;
    return NULL;
}

static int64_t *dup_arr(const int64_t *a, int64_t n)
{
    int64_t *r = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (r && n > 0) memcpy(r, a, (size_t)n * sizeof(int64_t));
    return r;
}

orc_type *orc_basic(int64_t size, int *err)
{
    orc_type *t;
    if (size <= 0) return fail(err, ORC_ERR_ARG);
    t = new_node(K_BASIC);
    if (!t) return fail(err, ORC_ERR_NOMEM);
    /* a basic type: one entry at displacement 0; its alignment is its size */
    t->size = size;
    t->lb = 0;
    t->ub = size;
    t->tlb = 0;
    t->tub = size;
    t->align = size;
    t->nent = 1;
    if (err) *err = ORC_OK;
    return t;
}

orc_type *orc_contiguous(int64_t n, orc_type *c, int *err)
{
    orc_type *t;
    if (n < 0 || !c) return fail(err, ORC_ERR_ARG);
    t = new_node(K_CONTIG);
    if (!t) return fail(err, ORC_ERR_NOMEM);
    t->n = n;
    t->child = c;
    retain(c);
    return finish(t, err);
}

static orc_type *make_vec(kind_t k, int64_t n, int64_t bl, int64_t stride, orc_type *c, int *err)
{
    orc_type *t;
    if (n < 0 || bl < 0 || !c) return fail(err, ORC_ERR_ARG);
    t = new_node(k);
    if (!t) return fail(err, ORC_ERR_NOMEM);
    t->n = n;
    t->bl = bl;
    t->stride = stride;
    t->child = c;
    retain(c);
    return finish(t, err);
}

orc_type *orc_vector(int64_t n, int64_t bl, int64_t stride, orc_type *c, int *err)
{
    return make_vec(K_VECTOR, n, bl, stride, c, err);
}

orc_type *orc_hvector(int64_t n, int64_t bl, int64_t stride_bytes, orc_type *c, int *err)
{
    return make_vec(K_HVECTOR, n, bl, stride_bytes, c, err);
}

static orc_type *make_idx(kind_t k, int64_t n, const int64_t *bl, int64_t bl1, const int64_t *disp,
                          orc_type *c, int *err)
{
    orc_type *t;
    int64_t i;
    if (n < 0 || !c || (n > 0 && !disp)) return fail(err, ORC_ERR_ARG);
    if (bl) {
        for (i = 0; i < n; i++)
            if (bl[i] < 0) return fail(err, ORC_ERR_ARG);
    } else if (bl1 < 0) {
        return fail(err, ORC_ERR_ARG);
    }
    t = new_node(k);
    if (!t) return fail(err, ORC_ERR_NOMEM);
    t->n = n;
    t->bls = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    t->disps = dup_arr(disp, n);
    if (!t->bls || !t->disps) {
        orc_release(t);
        return fail(err, ORC_ERR_NOMEM);
    }
    for (i = 0; i < n; i++) t->bls[i] = bl ? bl[i] : bl1;
    t->child = c;
    retain(c);
    return finish(t, err);
}

orc_type *orc_indexed(int64_t n, const int64_t *bl, const int64_t *disp, orc_type *c, int *err)
{
    if (n > 0 && !bl) return fail(err, ORC_ERR_ARG);
    return make_idx(K_INDEXED, n, bl, 0, disp, c, err);
}

orc_type *orc_hindexed(int64_t n, const int64_t *bl, const int64_t *disp_bytes, orc_type *c, int *err)
{
    if (n > 0 && !bl) return fail(err, ORC_ERR_ARG);
    return make_idx(K_HINDEXED, n, bl, 0, disp_bytes, c, err);
}

orc_type *orc_indexed_block(int64_t n, int64_t bl, const int64_t *disp, orc_type *c, int *err)
{
    return make_idx(K_INDEXED, n, NULL, bl, disp, c, err);
}

orc_type *orc_hindexed_block(int64_t n, int64_t bl, const int64_t *disp_bytes, orc_type *c, int *err)
{
    return make_idx(K_HINDEXED, n, NULL, bl, disp_bytes, c, err);
}

orc_type *orc_struct(int64_t n, const int64_t *bl, const int64_t *disp, orc_type *const *c, int *err)
{
    orc_type *t;
    int64_t i;
    if (n < 0 || (n > 0 && (!bl || !disp || !c))) return fail(err, ORC_ERR_ARG);
    for (i = 0; i < n; i++)
        if (bl[i] < 0 || !c[i]) return fail(err, ORC_ERR_ARG);
    t = new_node(K_STRUCT);
    if (!t) return fail(err, ORC_ERR_NOMEM);
    t->n = n;
    t->bls = dup_arr(bl, n);
    t->disps = dup_arr(disp, n);
    t->kids = (orc_type **)calloc((size_t)(n > 0 ? n : 1), sizeof(orc_type *));
    if (!t->bls || !t->disps || !t->kids) {
        t->n = 0;
        orc_release(t);
        return fail(err, ORC_ERR_NOMEM);
    }
    for (i = 0; i < n; i++) {
        t->kids[i] = c[i];
        retain(c[i]);
    }
    return finish(t, err);
}

orc_type *orc_subarray(int nd, const int64_t *sizes, const int64_t *subsizes, const int64_t *starts,
                       int order, orc_type *c, int *err)
{
    orc_type *t;
    int k;
    if (nd < 1 || nd > ORC_MAX_DIMS || !c || !sizes || !subsizes || !starts) return fail(err, ORC_ERR_ARG);
    if (order != ORC_ORDER_C && order != ORC_ORDER_FORTRAN) return fail(err, ORC_ERR_ARG);
    for (k = 0; k < nd; k++) {
        if (sizes[k] < 1 || subsizes[k] < 0 || starts[k] < 0) return fail(err, ORC_ERR_ARG);
        if (subsizes[k] > sizes[k] || starts[k] > sizes[k] - subsizes[k]) return fail(err, ORC_ERR_ARG);
    }
    t = new_node(K_SUBARRAY);
    if (!t) return fail(err, ORC_ERR_NOMEM);
    t->nd = nd;
    t->order = order;
    t->sizes = dup_arr(sizes, nd);
    t->subs = dup_arr(subsizes, nd);
    t->starts = dup_arr(starts, nd);
    if (!t->sizes || !t->subs || !t->starts) {
        orc_release(t);
        return fail(err, ORC_ERR_NOMEM);
    }
    t->child = c;
    retain(c);
    return finish(t, err);
}

/* Distributed array (MPI semantics): the elements of an nd-dimensional
 * global array that process `rank` of a row-major process grid owns.  Each
 * dimension's owned indices are found by asking, index by index, which grid
 * coordinate owns it: block distribution, owner = i / b (b = darg, or
 * ceil(g / p) by default); cyclic, owner = (i / k) mod p (k = darg, or 1);
 * none, the single coordinate 0. */
orc_type *orc_darray(int size, int rank, int nd, const int64_t *gsizes, const int *distribs, const int *dargs,
                     const int *psizes, int order, orc_type *c, int *err)
{
    orc_type *t;
    int64_t coord[ORC_MAX_DIMS], nproc = 1, total = 0, i;
    int k, r;
    if (nd < 1 || nd > ORC_MAX_DIMS || !c || !gsizes || !distribs || !dargs || !psizes) return fail(err, ORC_ERR_ARG);
    if (order != ORC_ORDER_C && order != ORC_ORDER_FORTRAN) return fail(err, ORC_ERR_ARG);
    if (size < 1 || rank < 0 || rank >= size) return fail(err, ORC_ERR_ARG);
    for (k = 0; k < nd; k++) {
        if (gsizes[k] < 1 || psizes[k] < 1 || !mul_ok(nproc, psizes[k], &nproc)) return fail(err, ORC_ERR_ARG);
        if (dargs[k] != ORC_DFLT_DARG && dargs[k] < 1) return fail(err, ORC_ERR_ARG);
        if (distribs[k] == ORC_DISTRIBUTE_NONE && psizes[k] != 1) return fail(err, ORC_ERR_ARG);
        if (distribs[k] == ORC_DISTRIBUTE_BLOCK && dargs[k] != ORC_DFLT_DARG &&
            (int64_t)dargs[k] * psizes[k] < gsizes[k])
            return fail(err, ORC_ERR_ARG);
        if (distribs[k] != ORC_DISTRIBUTE_NONE && distribs[k] != ORC_DISTRIBUTE_BLOCK &&
            distribs[k] != ORC_DISTRIBUTE_CYCLIC)
            return fail(err, ORC_ERR_ARG);
        if (!add_ok(total, gsizes[k], &total)) return fail(err, ORC_ERR_ARG);
    }
    if (nproc != size) return fail(err, ORC_ERR_ARG);
    r = rank;
    for (k = nd - 1; k >= 0; k--) {
        coord[k] = r % psizes[k];
        r /= psizes[k];
    }
    t = new_node(K_DARRAY);
    if (!t) return fail(err, ORC_ERR_NOMEM);
    t->nd = nd;
    t->order = order;
    t->sizes = dup_arr(gsizes, nd);
    t->own = (int64_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int64_t));
    t->own_off = (int64_t *)malloc((size_t)(nd + 1) * sizeof(int64_t));
    if (!t->sizes || !t->own || !t->own_off) {
        orc_release(t);
        return fail(err, ORC_ERR_NOMEM);
    }
    t->own_off[0] = 0;
    for (k = 0; k < nd; k++) {
        int64_t g = gsizes[k], p = psizes[k], n = t->own_off[k];
        int64_t b = dargs[k] == ORC_DFLT_DARG ? (distribs[k] == ORC_DISTRIBUTE_BLOCK ? (g + p - 1) / p : 1) : dargs[k];
        for (i = 0; i < g; i++) {
            int64_t owner = 0;
            if (distribs[k] == ORC_DISTRIBUTE_BLOCK) owner = i / b;
            else if (distribs[k] == ORC_DISTRIBUTE_CYCLIC) owner = (i / b) % p;
            if (owner == coord[k]) t->own[n++] = i;
        }
        t->own_off[k + 1] = n;
    }
    t->child = c;
    retain(c);
    return finish(t, err);
}

orc_type *orc_resized(orc_type *c, int64_t lb, int64_t extent, int *err)
{
    orc_type *t;
    if (!c) return fail(err, ORC_ERR_ARG);
    t = new_node(K_RESIZED);
    if (!t) return fail(err, ORC_ERR_NOMEM);
    t->rlb = lb;
    t->rext = extent;
    t->child = c;
    retain(c);
    return finish(t, err);
}

orc_type *orc_dup(orc_type *c, int *err)
{
    orc_type *t;
    if (!c) return fail(err, ORC_ERR_ARG);
    t = new_node(K_DUP);
    if (!t) return fail(err, ORC_ERR_NOMEM);
    t->child = c;
    retain(c);
    return finish(t, err);
}

int orc_attrs(const orc_type *t, int64_t out[8])
{
    if (!t || !out) return ORC_ERR_ARG;
    out[0] = t->size;
    out[1] = t->lb;
    out[2] = t->ub;
    out[3] = t->tlb;
    out[4] = t->tub;
    out[5] = t->align;
    out[6] = t->expl;
    out[7] = t->nent;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* the walk: every basic entry, in map order, as a byte run              */

typedef struct sink sink;
struct sink {
    /* called for each basic entry (addr, len) at packed position P;
     * returns nonzero to stop the walk */
    int (*run)(sink *s, int64_t addr, int64_t len);
    int64_t P;       /* packed bytes emitted so far */
    int64_t lo, hi;  /* packed range of interest (pack/unpack) */
    int skip;        /* skip whole copies that end before lo */
};

typedef struct {
    sink *s;
    int64_t base;
} emit_ctx;

static int emit(const orc_type *t, int64_t base, sink *s);

static int emit_cb(void *ctx, int64_t shift, const orc_type *c)
{
    emit_ctx *E = (emit_ctx *)ctx;
    return emit(c, E->base + shift, E->s);
}

static int emit(const orc_type *t, int64_t base, sink *s)
{
    emit_ctx E;
    if (t->size == 0) return 0;
    if (s->skip && s->P + t->size <= s->lo) {
        s->P += t->size;
        return 0;
    }
    if (t->kind == K_BASIC) return s->run(s, base, t->size);
    E.s = s;
    E.base = base;
    return for_each_copy(t, emit_cb, &E) != 0;
}

/* ------------------------------------------------------------------ */
/* segments: runs merged while each starts where the previous one ended */

typedef struct {
    sink s;
    int have;
    int64_t cur_base, cur_len;
    int64_t nseg;     /* finalized segments so far */
    int64_t prefix;   /* bytes in finalized segments */
    /* mode-specific */
    int mode;         /* 0 count all, 1 iov_len, 2 iov */
    int64_t max_bytes;
    int64_t off, m;
    int64_t *obase, *olen, got;
    int stop;
} seg_sink;

/* Finalize the current segment; returns nonzero to stop the walk. */
static int seg_finalize(seg_sink *S)
{
    if (S->mode == 1) {
        /* whole segments inside max_iov_bytes */
        if (S->prefix + S->cur_len > S->max_bytes) return 1;
    } else if (S->mode == 2) {
        if (S->nseg >= S->off + S->m) return 1;
        if (S->nseg >= S->off) {
            S->obase[S->got] = S->cur_base;
            S->olen[S->got] = S->cur_len;
            S->got++;
        }
    }
    S->nseg++;
    S->prefix += S->cur_len;
    return 0;
}

static int seg_run(sink *s, int64_t addr, int64_t len)
{
    seg_sink *S = (seg_sink *)s;
    if (S->have && S->cur_base + S->cur_len == addr) {
        S->cur_len += len;
        return 0;
    }
    if (S->have && seg_finalize(S)) {
        S->stop = 1;
        return 1;
    }
    S->have = 1;
    S->cur_base = addr;
    S->cur_len = len;
    return 0;
}

/* The segments of `count` consecutive elements: element r's typemap shifted
 * by r * extent, in order, through one merging sink, so a run that ends
 * where the next element's first run starts merges with it. */
static void seg_walk(const orc_type *t, int64_t count, seg_sink *S)
{
    S->s.run = seg_run;
    S->s.P = 0;
    S->s.lo = 0;
    S->s.hi = INT64_MAX;
    S->s.skip = 0;
    for (int64_t r = 0; r < count && !S->stop; r++) emit(t, r * (t->ub - t->lb), &S->s);
    if (!S->stop && S->have) seg_finalize(S);
}

/* count >= 0 and count * size, count * extent representable */
static int count_ok(const orc_type *t, int64_t count)
{
    int64_t x;
    if (count < 0) return 0;
    if (count > 0 && __builtin_mul_overflow(count, t->size, &x)) return 0;
    if (count > 0 && __builtin_mul_overflow(count, t->ub - t->lb, &x)) return 0;
    return 1;
}

int orc_num_segments_count(const orc_type *t, int64_t count, int64_t *nseg)
{
    seg_sink S;
    if (!t || !nseg || !count_ok(t, count)) return ORC_ERR_ARG;
    memset(&S, 0, sizeof S);
    S.mode = 0;
    seg_walk(t, count, &S);
    *nseg = S.nseg;
    return ORC_OK;
}

int orc_num_segments(const orc_type *t, int64_t *nseg) { return orc_num_segments_count(t, 1, nseg); }

int orc_iov_len_count(const orc_type *t, int64_t count, int64_t max_iov_bytes, int64_t *iov_len,
                      int64_t *actual_bytes)
{
    seg_sink S;
    if (!t || !iov_len || !actual_bytes || !count_ok(t, count)) return ORC_ERR_ARG;
    if (max_iov_bytes < -1) return ORC_ERR_ARG;
    memset(&S, 0, sizeof S);
    if (max_iov_bytes == -1 || max_iov_bytes > count * t->size) {
        /* all segments, all bytes */
        S.mode = 0;
        seg_walk(t, count, &S);
        *iov_len = S.nseg;
        *actual_bytes = count * t->size;
        return ORC_OK;
    }
    S.mode = 1;
    S.max_bytes = max_iov_bytes;
    seg_walk(t, count, &S);
    *iov_len = S.nseg;
    *actual_bytes = S.prefix;
    return ORC_OK;
}

int orc_iov_len(const orc_type *t, int64_t max_iov_bytes, int64_t *iov_len, int64_t *actual_bytes)
{
    return orc_iov_len_count(t, 1, max_iov_bytes, iov_len, actual_bytes);
}

int orc_iov_count(const orc_type *t, int64_t count, int64_t iov_offset, int64_t *base, int64_t *len,
                  int64_t max_iov_len, int64_t *actual_iov_len)
{
    seg_sink S;
    if (!t || !actual_iov_len || iov_offset < 0 || max_iov_len < 0 || !count_ok(t, count)) return ORC_ERR_ARG;
    if (max_iov_len > 0 && (!base || !len)) return ORC_ERR_ARG;
    memset(&S, 0, sizeof S);
    S.mode = 2;
    S.off = iov_offset;
    S.m = max_iov_len;
    S.obase = base;
    S.olen = len;
    if (max_iov_len > 0) seg_walk(t, count, &S);
    *actual_iov_len = S.got;
    return ORC_OK;
}

int orc_iov(const orc_type *t, int64_t iov_offset, int64_t *base, int64_t *len, int64_t max_iov_len,
            int64_t *actual_iov_len)
{
    return orc_iov_count(t, 1, iov_offset, base, len, max_iov_len, actual_iov_len);
}

/* ------------------------------------------------------------------ */
/* pack / unpack                                                        */

typedef struct {
    sink s;
    int unpack;
    uint8_t *origin_w;        /* unpack target */
    const uint8_t *origin_r;  /* pack source */
    const uint8_t *packed_r;  /* unpack source (packed byte lo at index 0) */
    uint8_t *packed_w;        /* pack target (packed byte lo at index 0) */
} copy_sink;

static int copy_run(sink *s, int64_t addr, int64_t len)
{
    copy_sink *C = (copy_sink *)s;
    int64_t a = s->P > s->lo ? s->P : s->lo;
    int64_t b = s->P + len < s->hi ? s->P + len : s->hi;
    if (a < b) {
        if (C->unpack)
            memcpy(C->origin_w + addr + (a - s->P), C->packed_r + (a - s->lo), (size_t)(b - a));
        else
            memcpy(C->packed_w + (a - s->lo), C->origin_r + addr + (a - s->P), (size_t)(b - a));
    }
    s->P += len;
    return s->P >= s->hi;
}

/* Walk elements r = 0 .. count-1 of the stream, each at r * extent. */
static void walk_count(const orc_type *t, int64_t count, copy_sink *C)
{
    int64_t r, E = extent_of(t);
    for (r = 0; r < count; r++) {
        if (C->s.P >= C->s.hi) break;
        if (emit(t, r * E, &C->s)) break;
    }
}

/* Validate count against the type: the stream length and every element
 * displacement must be representable. */
static int stream_total(const orc_type *t, int64_t count, int64_t *total)
{
    int64_t v;
    if (count < 0) return ORC_ERR_ARG;
    if (!mul_ok(count, t->size, total)) return ORC_ERR_ARG;
    if (count > 0) {
        int64_t w;
        if (!mul_ok(count - 1, extent_of(t), &v)) return ORC_ERR_ARG;
        if (!add_ok(v, t->tub, &w) || !add_ok(v, t->tlb, &w)) return ORC_ERR_ARG;
    }
    return ORC_OK;
}

int orc_pack(const uint8_t *origin, int64_t count, const orc_type *t, int64_t inoffset, uint8_t *out,
             int64_t max_pack_bytes, int64_t *actual)
{
    copy_sink C;
    int64_t total, n;
    int rc;
    if (!t || !actual || inoffset < 0 || max_pack_bytes < -1) return ORC_ERR_ARG;
    rc = stream_total(t, count, &total);
    if (rc) return rc;
    /* actual = clamp(total - inoffset, 0, max) */
    n = total - inoffset;
    if (n < 0) n = 0;
    if (max_pack_bytes >= 0 && n > max_pack_bytes) n = max_pack_bytes;
    *actual = n;
    if (n == 0) return ORC_OK;
    memset(&C, 0, sizeof C);
    C.s.run = copy_run;
    C.s.lo = inoffset;
    C.s.hi = inoffset + n;
    C.s.skip = 1;
    C.origin_r = origin;
    C.packed_w = out;
    walk_count(t, count, &C);
    return ORC_OK;
}

typedef struct {
    const uint8_t *origin;
    int64_t count;
    const orc_type *t;
    int64_t lo, hi;
    uint8_t *out;
    int64_t next;
    pthread_mutex_t mu;
} mt_job;

#define ORC_MT_CHUNK ((int64_t)1 << 20)

static void *mt_worker(void *arg)
{
    mt_job *J = (mt_job *)arg;
    for (;;) {
        int64_t k, a, n, got;
        pthread_mutex_lock(&J->mu);
        k = J->next++;
        pthread_mutex_unlock(&J->mu);
        a = J->lo + k * ORC_MT_CHUNK;
        if (a >= J->hi) break;
        n = J->hi - a < ORC_MT_CHUNK ? J->hi - a : ORC_MT_CHUNK;
        orc_pack(J->origin, J->count, J->t, a, J->out + (a - J->lo), n, &got);
    }
    return NULL;
}

int orc_pack_mt(const uint8_t *origin, int64_t count, const orc_type *t, int64_t inoffset, uint8_t *out,
                int64_t max_pack_bytes, int64_t *actual, int nthreads)
{
    int64_t total, n;
    int rc, i;
    mt_job J;
    pthread_t th[256];
    if (!t || !actual || inoffset < 0 || max_pack_bytes < -1 || nthreads < 1) return ORC_ERR_ARG;
    if (nthreads > 256) nthreads = 256;
    rc = stream_total(t, count, &total);
    if (rc) return rc;
    n = total - inoffset;
    if (n < 0) n = 0;
    if (max_pack_bytes >= 0 && n > max_pack_bytes) n = max_pack_bytes;
    *actual = n;
    if (n == 0) return ORC_OK;
    J.origin = origin;
    J.count = count;
    J.t = t;
    J.lo = inoffset;
    J.hi = inoffset + n;
    J.out = out;
    J.next = 0;
    pthread_mutex_init(&J.mu, NULL);
    for (i = 0; i < nthreads; i++) pthread_create(&th[i], NULL, mt_worker, &J);
    for (i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
    pthread_mutex_destroy(&J.mu);
    return ORC_OK;
}

/* --- overlap: does any byte belong to two entries of (count x t)? --- */

typedef struct {
    sink s;
    int64_t *addr, *len;
    int64_t n, cap;
    int nomem;
} list_sink;

static int list_run(sink *s, int64_t addr, int64_t len)
{
    list_sink *L = (list_sink *)s;
    if (L->n == L->cap) {
        int64_t nc = L->cap ? 2 * L->cap : 1024;
        int64_t *na = (int64_t *)realloc(L->addr, (size_t)nc * sizeof(int64_t));
        int64_t *nl;
        if (!na) { L->nomem = 1; return 1; }
        L->addr = na;
        nl = (int64_t *)realloc(L->len, (size_t)nc * sizeof(int64_t));
        if (!nl) { L->nomem = 1; return 1; }
        L->len = nl;
        L->cap = nc;
    }
    L->addr[L->n] = addr;
    L->len[L->n] = len;
    L->n++;
    return 0;
}

typedef struct {
    int64_t a, l;
} pair_t;

static int pair_cmp(const void *x, const void *y)
{
    const pair_t *p = (const pair_t *)x, *q = (const pair_t *)y;
    return (p->a > q->a) - (p->a < q->a);
}

static int has_overlap(const orc_type *t, int64_t count, int *overlap)
{
    list_sink L;
    pair_t *P;
    int64_t r, i, E = extent_of(t);
    memset(&L, 0, sizeof L);
    L.s.run = list_run;
    L.s.lo = 0;
    L.s.hi = INT64_MAX;
    for (r = 0; r < count && !L.nomem; r++) emit(t, r * E, &L.s);
    if (L.nomem) {
        free(L.addr);
        free(L.len);
        return ORC_ERR_NOMEM;
    }
    P = (pair_t *)malloc((size_t)(L.n > 0 ? L.n : 1) * sizeof(pair_t));
    if (!P) {
        free(L.addr);
        free(L.len);
        return ORC_ERR_NOMEM;
    }
    for (i = 0; i < L.n; i++) {
        P[i].a = L.addr[i];
        P[i].l = L.len[i];
    }
    free(L.addr);
    free(L.len);
    qsort(P, (size_t)L.n, sizeof(pair_t), pair_cmp);
    *overlap = 0;
    for (i = 0; i + 1 < L.n; i++)
        if (P[i].a + P[i].l > P[i + 1].a) {
            *overlap = 1;
            break;
        }
    free(P);
    return ORC_OK;
}

int orc_unpack(const uint8_t *in, int64_t insize, uint8_t *origin, int64_t count, const orc_type *t,
               int64_t outoffset, int64_t *actual)
{
    copy_sink C;
    int64_t total, remaining;
    int rc, ov = 0;
    if (!t || !actual || insize < 0 || outoffset < 0) return ORC_ERR_ARG;
    rc = stream_total(t, count, &total);
    if (rc) return rc;
    remaining = total - outoffset;
    if (remaining < 0) remaining = 0;
    if (insize > remaining) return ORC_ERR_TRUNCATE;
    rc = has_overlap(t, count, &ov);
    if (rc) return rc;
    if (ov) return ORC_ERR_OVERLAP;
    *actual = insize;
    if (insize == 0) return ORC_OK;
    memset(&C, 0, sizeof C);
    C.unpack = 1;
    C.s.run = copy_run;
    C.s.lo = outoffset;
    C.s.hi = outoffset + insize;
    C.s.skip = 1;
    C.origin_w = origin;
    C.packed_r = in;
    walk_count(t, count, &C);
    return ORC_OK;
}
