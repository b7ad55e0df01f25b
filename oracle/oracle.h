/*
 * oracle.h -- reference typemap walker for MPI-style derived datatypes.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plain CPU definition of what
 * the datatype extension computes (Derived Datatypes section: the segment
 * queries MPIX_Type_iov_len / MPIX_Type_iov and the MPIX_Iov layout), plus
 * the byte-stream pack/unpack that the typemap defines.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or helper with the product library;
 * it does not include include/mdt.h.
 *
 * Every type is an ordered typemap of (basic entry, byte displacement)
 * pairs.  The walker enumerates that map literally, copy by copy, in the
 * constructor's emission order, and derives every answer from it.
 *
 * Parity pinning: every function here is pinned by tests that do not call
 * it for their expected values (brute-force typemap lists, numpy slicing
 * and structured dtypes, closed forms of the worked example).
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_OK = 0,
    ORC_ERR_ARG = 1,      /* invalid argument (negative count, bad bounds, overflow) */
    ORC_ERR_OVERLAP = 2,  /* unpack target typemap has overlapping bytes */
    ORC_ERR_TRUNCATE = 3, /* unpack input longer than the remaining stream */
    ORC_ERR_NOMEM = 4
};

enum { ORC_ORDER_C = 0, ORC_ORDER_FORTRAN = 1 };

typedef struct orc_type orc_type;

/* Constructors.  Return NULL on invalid arguments (status in *err when
 * err != NULL).  Arrays are deep-copied.  Children are reference-counted;
 * the caller keeps its own reference and releases it with orc_release. */
orc_type *orc_basic(int64_t size, int *err);
orc_type *orc_contiguous(int64_t n, orc_type *c, int *err);
orc_type *orc_vector(int64_t n, int64_t bl, int64_t stride, orc_type *c, int *err);
orc_type *orc_hvector(int64_t n, int64_t bl, int64_t stride_bytes, orc_type *c, int *err);
orc_type *orc_indexed(int64_t n, const int64_t *bl, const int64_t *disp, orc_type *c, int *err);
orc_type *orc_hindexed(int64_t n, const int64_t *bl, const int64_t *disp_bytes, orc_type *c, int *err);
orc_type *orc_indexed_block(int64_t n, int64_t bl, const int64_t *disp, orc_type *c, int *err);
orc_type *orc_hindexed_block(int64_t n, int64_t bl, const int64_t *disp_bytes, orc_type *c, int *err);
orc_type *orc_struct(int64_t n, const int64_t *bl, const int64_t *disp_bytes, orc_type *const *c, int *err);
orc_type *orc_subarray(int nd, const int64_t *sizes, const int64_t *subsizes, const int64_t *starts,
                       int order, orc_type *c, int *err);
/* distributions of orc_darray */
#define ORC_DISTRIBUTE_NONE 0
#define ORC_DISTRIBUTE_BLOCK 1
#define ORC_DISTRIBUTE_CYCLIC 2
#define ORC_DFLT_DARG (-1)
orc_type *orc_darray(int size, int rank, int nd, const int64_t *gsizes, const int *distribs, const int *dargs,
                     const int *psizes, int order, orc_type *c, int *err);
orc_type *orc_resized(orc_type *c, int64_t lb, int64_t extent, int *err);
orc_type *orc_dup(orc_type *c, int *err);
void orc_release(orc_type *t);

/* Attributes: out[0..7] = size, lb, ub, true_lb, true_ub, align,
 * explicit_bounds, number of typemap entries. */
int orc_attrs(const orc_type *t, int64_t out[8]);

/* Segment queries (Derived Datatypes, Extension).  Segments are maximal
 * runs of typemap bytes that are contiguous both in memory and in map order;
 * base values are byte displacements from the buffer origin. */
int orc_num_segments(const orc_type *t, int64_t *nseg);
int orc_iov_len(const orc_type *t, int64_t max_iov_bytes, int64_t *iov_len, int64_t *actual_bytes);
int orc_iov(const orc_type *t, int64_t iov_offset, int64_t *base, int64_t *len, int64_t max_iov_len,
            int64_t *actual_iov_len);
/* The same queries over `count` consecutive elements (element r at r *
 * extent); a segment may then span an element boundary.  count = 1 is the
 * single-type form above; count = 0 has no segments. */
int orc_num_segments_count(const orc_type *t, int64_t count, int64_t *nseg);
int orc_iov_len_count(const orc_type *t, int64_t count, int64_t max_iov_bytes, int64_t *iov_len,
                      int64_t *actual_bytes);
int orc_iov_count(const orc_type *t, int64_t count, int64_t iov_offset, int64_t *base, int64_t *len,
                  int64_t max_iov_len, int64_t *actual_iov_len);

/* Pack bytes [inoffset, inoffset + actual) of the packed stream of
 * (count x t) read from `origin` into `out`; actual = clamp(count*size -
 * inoffset, 0, max) with max = -1 meaning unlimited. */
int orc_pack(const uint8_t *origin, int64_t count, const orc_type *t, int64_t inoffset, uint8_t *out,
             int64_t max_pack_bytes, int64_t *actual);
/* Same, split into 1 MiB byte ranges processed by `nthreads` threads. */
int orc_pack_mt(const uint8_t *origin, int64_t count, const orc_type *t, int64_t inoffset, uint8_t *out,
                int64_t max_pack_bytes, int64_t *actual, int nthreads);
/* Inverse: write packed bytes [outoffset, outoffset + insize) of the stream
 * of (count x t) into `origin`.  Gaps are never written. */
int orc_unpack(const uint8_t *in, int64_t insize, uint8_t *origin, int64_t count, const orc_type *t,
               int64_t outoffset, int64_t *actual);

#ifdef __cplusplus
}
#endif
#endif
