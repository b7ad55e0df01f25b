/*
 * mdt.h -- C ABI of libmdt: MPI-style derived datatypes on MI355X (gfx950).
 *
 * What it implements (arXiv 2402.12274, "Designing and Prototyping
 * Extensions to MPI in MPICH"):
 *   - Derived Datatypes section: datatypes as a nested, offset, possibly
 *     overlapping memory-layout description, and the extension that lets a
 *     user read a committed datatype's segments as an iovec list
 *     (MPIX_Type_iov_len, MPIX_Type_iov, MPIX_Iov).  mdt_type_iov_len and
 *     mdt_type_iov are those two calls; mdt_iov is MPIX_Iov.
 *   - The gather/scatter that such a layout drives: pack and unpack of
 *     device-resident buffers, by byte range of the packed stream (General
 *     Progress, Background: large messages move as pipelined chunks).
 *   - Offloading Asynchronous Operations section: work enqueued on a GPU
 *     stream runs in that stream's order; starting it and waiting for it
 *     are separate host-side steps (mdt_*_enqueue, mdt_wait, mdt_test).
 *   - MPIX Streams / General Progress sections: a stream is a serial
 *     execution context; progress can be driven explicitly or by a progress
 *     thread (mdt_server_progress, mdt_server_start_progress_thread).
 *
 * Conventions (apply to every call):
 *   - Every call returns MDT_SUCCESS (0) or an MDT_ERR_* code.  On error no
 *     output argument is written and no device work is enqueued.
 *   - Counts, sizes, displacements and offsets are int64 (mdt_count,
 *     mdt_aint).  Displacements may be negative.
 *   - Buffer arguments of pack/unpack are *device* pointers (memory from
 *     hipMalloc or a framework allocator on the current HIP device) unless
 *     stated otherwise.  They are owned by the caller and must stay valid
 *     until the work that uses them has completed.
 *   - A buffer "origin" is the address of displacement 0 of element 0; the
 *     typemap's bytes of element r sit at origin + r*extent + displacement.
 *   - Offsets and budgets of pack/unpack are byte positions in the packed
 *     stream of (count x type).  Partial ranges may split basic elements.
 *   - Type handles are reference counted: constructors deep-copy their
 *     array arguments and hold references to their children, so freeing a
 *     type never invalidates a type built from it.
 *   - Threads: type construction, commit and queries are thread safe.  An
 *     mdt_stream is a serial context: concurrent calls on one stream are a
 *     caller error; different streams never contend.
 */
#ifndef MDT_H
#define MDT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define MDT_API __attribute__((visibility("default")))
#else
#define MDT_API
#endif

typedef int64_t mdt_count; /* MPI_Count */
typedef int64_t mdt_aint;  /* MPI_Aint */

typedef struct mdt_type_s *mdt_type;
typedef struct mdt_stream_s *mdt_stream;
typedef struct mdt_request_s *mdt_request;
typedef struct mdt_batch_s *mdt_batch;
typedef struct mdt_server_s *mdt_server;
/* Same layout as hipStream_t; kept opaque so this header needs no HIP headers. */
typedef struct ihipStream_t *mdt_hip_stream;

#define MDT_TYPE_NULL ((mdt_type)0)
#define MDT_REQUEST_NULL ((mdt_request)0)

/* MPIX_Iov: {base, len}; same layout as struct iovec (Derived Datatypes,
 * Extension).  Host queries store the segment's byte displacement from the
 * buffer origin in iov_base (it may be "negative"); the device flatten call
 * adds a caller-given base address. */
typedef struct mdt_iov {
    void *iov_base;
    mdt_aint iov_len;
} mdt_iov;

enum {
    MDT_SUCCESS = 0,
    MDT_ERR_ARG = 1,      /* invalid argument: negative count, bad bounds, overflow, NULL output */
    MDT_ERR_TYPE = 2,     /* NULL, freed or (where required) uncommitted type handle */
    MDT_ERR_COUNT = 3,    /* count out of range for the type (stream length overflows) */
    MDT_ERR_TRUNCATE = 4, /* unpack input longer than the remaining packed stream */
    MDT_ERR_OVERLAP = 5,  /* unpack target layout has overlapping bytes */
    MDT_ERR_NO_MEM = 6,   /* host or device allocation failed, or a size limit was hit */
    MDT_ERR_HIP = 7,      /* a HIP runtime call failed; see mdt_last_hip_error */
    MDT_ERR_AGAIN = 8,    /* non-blocking submit: admission budget currently full */
    MDT_ERR_STATE = 9     /* call not valid in the object's current state */
};

/* Predefined (basic) types.  A basic type has one entry at displacement 0;
 * its size, extent and alignment are all equal to its byte size. */
enum {
    MDT_CODE_BYTE = 0, MDT_CODE_CHAR, MDT_CODE_INT8, MDT_CODE_UINT8,
    MDT_CODE_INT16, MDT_CODE_UINT16, MDT_CODE_INT32, MDT_CODE_UINT32,
    MDT_CODE_INT, MDT_CODE_FLOAT, MDT_CODE_INT64, MDT_CODE_UINT64,
    MDT_CODE_DOUBLE, MDT_NUM_BASIC
};
/* Returns the (never freed, already committed) handle of a predefined type,
 * or MDT_TYPE_NULL for an unknown code. */
MDT_API mdt_type mdt_basic(int code);
#define MDT_BYTE mdt_basic(MDT_CODE_BYTE)
#define MDT_CHAR mdt_basic(MDT_CODE_CHAR)
#define MDT_INT8 mdt_basic(MDT_CODE_INT8)
#define MDT_UINT8 mdt_basic(MDT_CODE_UINT8)
#define MDT_INT16 mdt_basic(MDT_CODE_INT16)
#define MDT_UINT16 mdt_basic(MDT_CODE_UINT16)
#define MDT_INT32 mdt_basic(MDT_CODE_INT32)
#define MDT_UINT32 mdt_basic(MDT_CODE_UINT32)
#define MDT_INT mdt_basic(MDT_CODE_INT)
#define MDT_FLOAT mdt_basic(MDT_CODE_FLOAT)
#define MDT_INT64 mdt_basic(MDT_CODE_INT64)
#define MDT_UINT64 mdt_basic(MDT_CODE_UINT64)
#define MDT_DOUBLE mdt_basic(MDT_CODE_DOUBLE)

enum { MDT_ORDER_C = 0, MDT_ORDER_FORTRAN = 1 };

/* ---------------------------------------------------------------------
 * Type constructors (Derived Datatypes: nested layouts with offsets; the
 * worked example builds a contiguous type and a subarray of it).  Each
 * follows the MPI constructor of the same name; E below is the extent of
 * the child type.  *out receives a new, uncommitted handle.
 *   contiguous(n, c):            copy i at i*E, i < n
 *   vector(n, bl, stride, c):    copy (i, j) at (i*stride + j)*E
 *   hvector(n, bl, stride, c):   copy (i, j) at i*stride + j*E  (stride in bytes)
 *   indexed(n, bl[], disp[], c): copy (i, j) at (disp[i] + j)*E, j < bl[i]
 *   hindexed(...):               copy (i, j) at disp[i] + j*E   (disp in bytes)
 *   *_block: the same with one block length for all blocks
 *   struct(n, bl[], disp[], c[]): copy (i, j) of c[i] at disp[i] + j*extent(c[i]);
 *       the extent is padded up to a multiple of the largest member
 *       alignment unless a member has explicit bounds (resized/subarray)
 *   subarray(nd, sizes, subsizes, starts, order, c): the sub-box of an
 *       nd-dimensional array of c, row-major (C) or column-major (Fortran);
 *       lb = 0, extent = prod(sizes)*E.  subsizes may be 0 (empty type).
 *   resized(c, lb, extent): the typemap of c with the given bounds
 *   dup(c): the same typemap and bounds
 * Errors: MDT_ERR_ARG for negative counts/lengths, invalid subarray bounds,
 * NULL arrays with n > 0, or 64-bit overflow of any displacement or bound;
 * MDT_ERR_TYPE for an invalid child handle. */
MDT_API int mdt_type_contiguous(mdt_count n, mdt_type old, mdt_type *out);
MDT_API int mdt_type_vector(mdt_count n, mdt_count bl, mdt_count stride, mdt_type old, mdt_type *out);
MDT_API int mdt_type_create_hvector(mdt_count n, mdt_count bl, mdt_aint stride_bytes, mdt_type old,
                                    mdt_type *out);
MDT_API int mdt_type_indexed(mdt_count n, const mdt_count bl[], const mdt_count disp[], mdt_type old,
                             mdt_type *out);
MDT_API int mdt_type_create_hindexed(mdt_count n, const mdt_count bl[], const mdt_aint disp[], mdt_type old,
                                     mdt_type *out);
MDT_API int mdt_type_create_indexed_block(mdt_count n, mdt_count bl, const mdt_count disp[], mdt_type old,
                                          mdt_type *out);
MDT_API int mdt_type_create_hindexed_block(mdt_count n, mdt_count bl, const mdt_aint disp[], mdt_type old,
                                           mdt_type *out);
MDT_API int mdt_type_create_struct(mdt_count n, const mdt_count bl[], const mdt_aint disp[],
                                   const mdt_type types[], mdt_type *out);
MDT_API int mdt_type_create_subarray(int ndims, const mdt_count sizes[], const mdt_count subsizes[],
                                     const mdt_count starts[], int order, mdt_type old, mdt_type *out);
MDT_API int mdt_type_create_resized(mdt_type old, mdt_aint lb, mdt_aint extent, mdt_type *out);
MDT_API int mdt_type_dup(mdt_type old, mdt_type *out);

/* Distributed array (the constructor set the Derived Datatypes section
 * relies on, as in MPI): the part of an nd-dimensional global array of
 * `old` (sizes gsizes[], C or Fortran order) that process `rank` of a
 * size-process grid owns.  The grid has psizes[k] processes along
 * dimension k (their product is size) and ranks are laid out row-major
 * over it.  Along dimension k the process at grid coordinate p owns:
 *   MDT_DISTRIBUTE_NONE:   every index (psizes[k] must be 1);
 *   MDT_DISTRIBUTE_BLOCK:  [p*b, min((p+1)*b, g)), b = dargs[k], or
 *                          ceil(g / psizes[k]) for MDT_DISTRIBUTE_DFLT_DARG
 *                          (b * psizes[k] >= g is required);
 *   MDT_DISTRIBUTE_CYCLIC: the indices i with (i / k) mod psizes[k] == p,
 *                          k = dargs[k], or 1 for MDT_DISTRIBUTE_DFLT_DARG.
 * The typemap lists the owned elements in the array's order (last
 * dimension fastest for C, first for Fortran), element i at
 * linear(i) * extent(old); lb = 0, extent = prod(gsizes) * extent(old).
 * Errors: MDT_ERR_ARG for an invalid grid, rank, distribution or
 * argument, or 64-bit overflow. */
enum { MDT_DISTRIBUTE_NONE = 0, MDT_DISTRIBUTE_BLOCK = 1, MDT_DISTRIBUTE_CYCLIC = 2 };
#define MDT_DISTRIBUTE_DFLT_DARG (-1)
MDT_API int mdt_type_create_darray(int size, int rank, int ndims, const mdt_count gsizes[], const int distribs[],
                                   const int dargs[], const int psizes[], int order, mdt_type old,
                                   mdt_type *out);

/* Type envelope and contents (MPI_Type_get_envelope / get_contents: the
 * constructor call a type was made with, so a type can be described,
 * serialized and rebuilt).  The envelope gives the combiner and the lengths
 * of the three argument lists; the contents fill them:
 *   NAMED (a predefined type): no contents (get_contents: MDT_ERR_ARG)
 *   DUP:            types {old}
 *   CONTIGUOUS:     ints {count}; types {old}
 *   VECTOR:         ints {count, blocklength, stride}; types {old}
 *   HVECTOR:        ints {count, blocklength}; addrs {stride}; types {old}
 *   INDEXED:        ints {count, bl[count], disp[count]}; types {old}
 *   HINDEXED:       ints {count, bl[count]}; addrs {disp[count]}; types {old}
 *   INDEXED_BLOCK:  ints {count, blocklength, disp[count]}; types {old}
 *   HINDEXED_BLOCK: ints {count, blocklength}; addrs {disp[count]}; types {old}
 *   STRUCT:         ints {count, bl[count]}; addrs {disp[count]}; types[count]
 *   SUBARRAY:       ints {ndims, sizes[], subsizes[], starts[], order}; types {old}
 *   DARRAY:         ints {size, rank, ndims, gsizes[], distribs[], dargs[],
 *                   psizes[], order}; types {old}
 *   RESIZED:        addrs {lb, extent}; types {old}
 * Returned derived types are new references (release each with
 * mdt_type_free); predefined ones are returned as themselves.  Errors:
 * MDT_ERR_ARG if a max_* is below the envelope's count (nothing written). */
enum {
    MDT_COMBINER_NAMED = 0, MDT_COMBINER_DUP, MDT_COMBINER_CONTIGUOUS, MDT_COMBINER_VECTOR, MDT_COMBINER_HVECTOR,
    MDT_COMBINER_INDEXED, MDT_COMBINER_HINDEXED, MDT_COMBINER_INDEXED_BLOCK, MDT_COMBINER_HINDEXED_BLOCK,
    MDT_COMBINER_STRUCT, MDT_COMBINER_SUBARRAY, MDT_COMBINER_DARRAY, MDT_COMBINER_RESIZED
};
MDT_API int mdt_type_get_envelope(mdt_type t, mdt_count *num_integers, mdt_count *num_addresses,
                                  mdt_count *num_datatypes, int *combiner);
MDT_API int mdt_type_get_contents(mdt_type t, mdt_count max_integers, mdt_count max_addresses,
                                  mdt_count max_datatypes, mdt_count integers[], mdt_aint addresses[],
                                  mdt_type datatypes[]);

/* Commit (worked example: committed before it is queried): compiles the
 * layout program and uploads its tables to the current HIP device, where
 * they stay resident until the last reference is freed.  Committing twice
 * is a no-op.  Without a GPU the host layout is still built (queries work);
 * device tables are then uploaded on first device use. */
MDT_API int mdt_type_commit(mdt_type *t);
/* Release the caller's reference and set *t = MDT_TYPE_NULL.  Predefined
 * handles are not freed (MDT_ERR_TYPE).  The device tables of the type are
 * released when no type refers to it any more; their release waits for the
 * device to be idle. */
MDT_API int mdt_type_free(mdt_type *t);

/* Layout program summary of a committed type (not part of the paper's
 * interface: it reports which of this library's kernels a full transfer of
 * the type takes, for tests and tuning).
 *   kind:          0 empty, 1 contiguous, 2 one shape (loops over a run
 *                  list), 3 group table (irregular)
 *   groups, runs:  groups of the table (1 for kinds 1-2), runs of one element
 *   records:       1 when the stream is read as equally spaced records of
 *                  short runs (LDS-staged record kernels), else 0
 *   record_bytes, record_stride: packed bytes and byte stride of a record
 *   pack_table:    0 none, 1 per-byte table, 2 per-chunk table (records)
 *   unpack_table:  0 none (unpack takes the chunk path), 1 per-byte table,
 *                  2 per-dword table (records)
 *   device_bytes:  size of the type's resident device tables
 * Errors: MDT_ERR_TYPE for an invalid or uncommitted handle, MDT_ERR_ARG
 * for a NULL out. */
typedef struct mdt_layout_info {
    int32_t kind;
    int32_t records;
    int64_t groups;
    int64_t runs;
    int64_t record_bytes;
    int64_t record_stride;
    int32_t pack_table;
    int32_t unpack_table;
    int64_t device_bytes;
} mdt_layout_info;
MDT_API int mdt_type_layout_info(mdt_type t, mdt_layout_info *out);

/* Attributes (valid on uncommitted types). */
MDT_API int mdt_type_size(mdt_type t, mdt_count *size);
MDT_API int mdt_type_get_extent(mdt_type t, mdt_aint *lb, mdt_aint *extent);
MDT_API int mdt_type_get_true_extent(mdt_type t, mdt_aint *true_lb, mdt_aint *true_extent);

/* MPIX_Type_iov_len (Derived Datatypes, Extension).  Segments are maximal
 * runs of the type's bytes that are contiguous in memory and consecutive in
 * map order.  If max_iov_bytes is -1 or greater than the type size,
 * *iov_len = number of segments and *actual_iov_bytes = size; otherwise
 * *iov_len = number of whole leading segments whose bytes fit in
 * max_iov_bytes, and *actual_iov_bytes = their bytes (so P_k <= max <
 * P_{k+1}: the call bisects byte offsets to segment indices).  Other
 * negative values: MDT_ERR_ARG.  Requires a committed type. */
MDT_API int mdt_type_iov_len(mdt_type t, mdt_count max_iov_bytes, mdt_count *iov_len,
                             mdt_count *actual_iov_bytes);
/* MPIX_Type_iov: segments [iov_offset, iov_offset + max_iov_len) into the
 * caller-allocated host array iov; *actual_iov_len = how many were written
 * (0 when iov_offset >= number of segments).  iov_base holds the segment's
 * byte displacement from the origin, cast to a pointer. */
MDT_API int mdt_type_iov(mdt_type t, mdt_count iov_offset, mdt_iov *iov, mdt_count max_iov_len,
                         mdt_count *actual_iov_len);

/* The same two queries over count consecutive elements (Derived Datatypes,
 * Extension: the queries are stated for one datatype; this is the form for
 * a buffer of count elements, element r at r * extent).  Segments are those
 * of the count-fold typemap, merged where they touch, so an element's last
 * segment merges with the next element's first when it ends where that one
 * starts (the layout of contiguous(count, t)).  count = 1 is
 * mdt_type_iov_len / mdt_type_iov; count = 0 has no segments.  max_iov_bytes
 * is compared with count * size.  Errors: MDT_ERR_ARG for count < 0,
 * MDT_ERR_COUNT when count * size, count * extent or the segment count
 * overflows. */
MDT_API int mdt_type_iov_len_count(mdt_type t, mdt_count count, mdt_count max_iov_bytes, mdt_count *iov_len,
                                   mdt_count *actual_iov_bytes);
MDT_API int mdt_type_iov_count(mdt_type t, mdt_count count, mdt_count iov_offset, mdt_iov *iov,
                               mdt_count max_iov_len, mdt_count *actual_iov_len);

/* Blocking pack of bytes [inoffset, inoffset + actual) of the packed stream
 * of (incount x t) read from device buffer inbuf (the origin) into device
 * buffer outbuf; actual = clamp(incount*size - inoffset, 0, max_pack_bytes),
 * max_pack_bytes = -1 meaning unlimited.  The work runs on the null stream
 * and the call returns when it has completed.  Overlapping types pack. */
MDT_API int mdt_pack(const void *inbuf, mdt_count incount, mdt_type t, mdt_count inoffset, void *outbuf,
                     mdt_count max_pack_bytes, mdt_count *actual_pack_bytes);
/* Blocking unpack: writes the insize packed bytes at inbuf into stream
 * positions [outoffset, outoffset + insize) of (outcount x t) at origin
 * outbuf.  Bytes outside the typemap are never written.  Errors:
 * MDT_ERR_TRUNCATE if insize > outcount*size - outoffset, MDT_ERR_OVERLAP
 * if (outcount x t) has overlapping bytes.  *actual_unpack_bytes = insize. */
MDT_API int mdt_unpack(const void *inbuf, mdt_count insize, void *outbuf, mdt_count outcount, mdt_type t,
                       mdt_count outoffset, mdt_count *actual_unpack_bytes);

/* Blocking typed copy (Derived Datatypes: a typemap describes the layout on
 * each side of a transfer; this is the transfer to oneself, as a send and a
 * matching receive with different types): byte p of the packed stream of
 * (srccount x srctype) at origin src goes to stream position p of
 * (dstcount x dsttype) at origin dst, for p in [offset, offset + actual),
 * actual = clamp(srccount*srcsize - offset, 0, max_bytes) (max_bytes = -1:
 * unlimited), in one pass with no packed staging buffer.  Bytes of dst
 * outside its typemap are never written.  The bytes read and the bytes
 * written must not overlap.  Errors: MDT_ERR_TRUNCATE if actual >
 * dstcount*dstsize - offset, MDT_ERR_OVERLAP if (dstcount x dsttype) has
 * overlapping bytes; nothing is written on error. */
MDT_API int mdt_typed_copy(const void *src, mdt_count srccount, mdt_type srctype, void *dst, mdt_count dstcount,
                           mdt_type dsttype, mdt_count offset, mdt_count max_bytes, mdt_count *actual);

/* ---------------------------------------------------------------------
 * Stream-ordered work (Offloading Asynchronous Operations: work enqueued
 * on a GPU stream runs after earlier work on that stream and before later
 * work; the host starts it and waits for it separately). */
/* Wrap a caller-owned HIP stream (NULL = the null stream).  The library
 * never destroys the HIP stream. */
MDT_API int mdt_stream_create(mdt_hip_stream s, mdt_stream *out);
MDT_API int mdt_stream_free(mdt_stream *s);
/* As mdt_pack / mdt_unpack, but enqueued on stream s; the call returns
 * immediately (the actual byte count is known from sizes alone).  If req is
 * not NULL it receives a request that completes with the work. */
MDT_API int mdt_pack_enqueue(const void *inbuf, mdt_count incount, mdt_type t, mdt_count inoffset,
                             void *outbuf, mdt_count max_pack_bytes, mdt_count *actual_pack_bytes,
                             mdt_stream s, mdt_request *req);
MDT_API int mdt_unpack_enqueue(const void *inbuf, mdt_count insize, void *outbuf, mdt_count outcount,
                               mdt_type t, mdt_count outoffset, mdt_count *actual_unpack_bytes,
                               mdt_stream s, mdt_request *req);
/* As mdt_typed_copy, enqueued on stream s. */
MDT_API int mdt_typed_copy_enqueue(const void *src, mdt_count srccount, mdt_type srctype, void *dst,
                                   mdt_count dstcount, mdt_type dsttype, mdt_count offset, mdt_count max_bytes,
                                   mdt_count *actual, mdt_stream s, mdt_request *req);
/* Device flatten: write segments [iov_offset, iov_offset + max_iov_len) of
 * committed type t into the device array dev_iov, each base being
 * `base` + displacement (base may be NULL for raw displacements); enqueued
 * on s.  *actual_iov_len is returned immediately. */
MDT_API int mdt_type_iov_enqueue(mdt_type t, mdt_count iov_offset, mdt_iov *dev_iov, mdt_count max_iov_len,
                                 const void *base, mdt_count *actual_iov_len, mdt_stream s, mdt_request *req);
/* Device flatten of the count form (mdt_type_iov_count's segments). */
MDT_API int mdt_type_iov_count_enqueue(mdt_type t, mdt_count count, mdt_count iov_offset, mdt_iov *dev_iov,
                                       mdt_count max_iov_len, const void *base, mdt_count *actual_iov_len,
                                       mdt_stream s, mdt_request *req);
/* Complete a request (from an enqueue or batch launch, or a generalized
 * request): mdt_wait blocks; mdt_test sets *flag = 1 and frees the request
 * if it has completed, else *flag = 0.  Completed requests are freed and
 * set to MDT_REQUEST_NULL; a NULL request counts as complete.  mdt_waitall
 * completes all n (NULL entries allowed), driving generalized requests
 * together (one wait_fn call per group that shares it); on an error it
 * returns the first error and leaves the requests it did not complete
 * valid.  Server requests have their own calls (MDT_ERR_ARG here). */
MDT_API int mdt_wait(mdt_request *req);
MDT_API int mdt_test(mdt_request *req, int *flag);
MDT_API int mdt_waitall(int n, mdt_request reqs[]);

/* ---------------------------------------------------------------------
 * Generalized requests (Generalized Requests section and its extension
 * with poll and wait callbacks): a request for an asynchronous task the
 * caller runs itself (its own kernel, I/O), completed by the same mdt_test,
 * mdt_wait and mdt_waitall as the library's requests, with no progress
 * thread of the caller's.  extra_state is the caller's and is passed to
 * every callback; any callback may be NULL.
 *   poll_fn(extra_state): called by mdt_test, mdt_wait and mdt_waitall an
 *     unspecified number of times until the request is complete; it checks
 *     the task and calls mdt_grequest_complete once the task has finished.
 *   wait_fn(count, states, timeout): used by mdt_wait and mdt_waitall
 *     instead of repeated polls, with the states of the incomplete requests
 *     given to that call that share this wait_fn (in the order given); it
 *     blocks until those tasks have finished or timeout seconds have passed
 *     (timeout < 0: no limit), calling mdt_grequest_complete for each
 *     finished task.  mdt_test uses poll_fn only.
 *   query_fn(extra_state), then free_fn(extra_state): called once each when
 *     a completion call returns the completed request (and frees it).
 *   cancel_fn(extra_state, complete): called by mdt_cancel; complete is 1
 *     when mdt_grequest_complete has already been called.
 * A nonzero value returned by poll_fn or wait_fn ends the completion call
 * with that value and leaves the request incomplete and valid; a nonzero
 * value of query_fn or free_fn is returned by the completion call that
 * freed the request.  With neither poll_fn nor wait_fn the task itself
 * calls mdt_grequest_complete (from any thread) and mdt_wait blocks until
 * it has.  Callbacks must not complete (test, wait) their own request. */
typedef int (*mdt_grequest_query_fn)(void *extra_state);
typedef int (*mdt_grequest_free_fn)(void *extra_state);
typedef int (*mdt_grequest_cancel_fn)(void *extra_state, int complete);
typedef int (*mdt_grequest_poll_fn)(void *extra_state);
typedef int (*mdt_grequest_wait_fn)(int count, void *const *array_of_states, double timeout);
MDT_API int mdt_grequest_start(mdt_grequest_query_fn query_fn, mdt_grequest_free_fn free_fn,
                               mdt_grequest_cancel_fn cancel_fn, mdt_grequest_poll_fn poll_fn,
                               mdt_grequest_wait_fn wait_fn, void *extra_state, mdt_request *req);
/* Mark a generalized request's task finished (thread safe).  MDT_ERR_STATE
 * if it was already marked, MDT_ERR_ARG if req is not a generalized
 * request. */
MDT_API int mdt_grequest_complete(mdt_request req);
/* Cancel a generalized request: returns its cancel_fn's value (0 without
 * one); the request must still be completed by mdt_test or mdt_wait.  Work
 * enqueued on the GPU cannot be cancelled: MDT_ERR_ARG for other requests. */
MDT_API int mdt_cancel(mdt_request req);

/* ---------------------------------------------------------------------
 * General progress (General Progress section: progress invoked on its own,
 * not through a particular request, per stream, and a progress thread the
 * caller starts and stops around the phases that need it).
 *   mdt_stream_progress(s): one progress pass over the requests of work
 *     enqueued on stream s (mdt_*_enqueue, mdt_batch_launch,
 *     mdt_type_iov_enqueue with a request): each one whose work has
 *     finished is recorded as complete, so mdt_request_get_status reports
 *     it and mdt_test completes it without another runtime query.  s = NULL
 *     is general progress: every stream's requests and every generalized
 *     request, whose poll_fn is called (poll_fn is never called by two
 *     threads at once).  Returns the first error a pass met (a HIP error,
 *     or a poll_fn's nonzero value); the pass still visits every request.
 *   mdt_start_progress_thread(s) / mdt_stop_progress_thread(s): a library
 *     thread making such passes on s (NULL: general progress) back to back
 *     while some of its requests are incomplete and every 50 us otherwise;
 *     stop joins it.  Starting a running thread, or stopping a stopped one,
 *     does nothing.  mdt_stream_free stops the stream's thread; requests of
 *     a freed stream stay valid for mdt_test / mdt_wait.
 *   mdt_request_get_status(req, flag): *flag = 1 if req is known to be
 *     complete (an event request seen finished by a progress pass or a
 *     test; a generalized request marked by mdt_grequest_complete), without
 *     invoking progress and without freeing it.  Server requests have their
 *     own calls (MDT_ERR_ARG). */
MDT_API int mdt_stream_progress(mdt_stream s);
MDT_API int mdt_start_progress_thread(mdt_stream s);
MDT_API int mdt_stop_progress_thread(mdt_stream s);
MDT_API int mdt_request_get_status(mdt_request req, int *flag);

/* ---------------------------------------------------------------------
 * Batches: many pack/unpack requests of mixed types and sizes executed by
 * one kernel launch per direction (pack requests and copies first, then
 * unpack requests).  How that launch runs is the batch's configuration
 * (mdt_batch_config below): a persistent grid or one workgroup per tile,
 * each either launched directly or captured once in a HIP graph and
 * replayed; mdt_batch_autotune picks among them by timing the batch, and
 * mdt_batch_get_config reports the choice.  Requests are described on the
 * host; mdt_batch_launch uploads the descriptors (in stream order, only
 * when the batch changed) and runs them.  Every request's bytes are
 * identical to the same request run alone.  Destinations of different
 * requests must not overlap, except where the overlapping bytes receive
 * equal values (the faces of one array unpacked from one exchange meet
 * along their edges): the writes are byte-exact, so their order does not
 * matter then.  A batch may be launched on any stream: a
 * launch on a different stream than the batch's previous launch waits on
 * the device for that launch first (the batch's device-side descriptors
 * are shared by its launches). */
MDT_API int mdt_batch_create(mdt_batch *b);
MDT_API int mdt_batch_free(mdt_batch *b);
/* Remove all requests (the batch and its captured graph are reused). */
MDT_API int mdt_batch_clear(mdt_batch b);
MDT_API int mdt_batch_add_pack(mdt_batch b, const void *inbuf, mdt_count incount, mdt_type t,
                               mdt_count inoffset, void *outbuf, mdt_count max_pack_bytes,
                               mdt_count *actual_pack_bytes);
MDT_API int mdt_batch_add_unpack(mdt_batch b, const void *inbuf, mdt_count insize, void *outbuf,
                                 mdt_count outcount, mdt_type t, mdt_count outoffset,
                                 mdt_count *actual_unpack_bytes);
/* A typed copy (as mdt_typed_copy) as a request of the batch: it runs in the
 * first launch, with the pack requests; unpack requests run after it. */
MDT_API int mdt_batch_add_copy(mdt_batch b, const void *src, mdt_count srccount, mdt_type srctype, void *dst,
                               mdt_count dstcount, mdt_type dsttype, mdt_count offset, mdt_count max_bytes,
                               mdt_count *actual);
/* A relay (the two sides of a transfer through a staging buffer, General
 * Progress, Background: a message is packed for sending and unpacked where it
 * lands): bytes [offset, offset + actual) of the packed stream of (srccount
 * x srctype) at src are packed into the device buffer packed (as
 * mdt_batch_add_pack) and the same bytes are unpacked from it into the same
 * stream positions of (dstcount x dsttype) at dst (as mdt_batch_add_unpack),
 * actual = clamp(srccount*srcsize - offset, 0, max_bytes).  Both results
 * are those of the pack and the unpack run one after the other; in the
 * batch a workgroup unpacks each tile right after packing it, so the
 * packed bytes are read back from the cache and the pair costs one launch.
 * It runs in the first launch, with the pack requests.  Errors as
 * mdt_typed_copy; the packed buffer must not overlap src or dst. */
MDT_API int mdt_batch_add_relay(mdt_batch b, const void *src, mdt_count srccount, mdt_type srctype, void *packed,
                                void *dst, mdt_count dstcount, mdt_type dsttype, mdt_count offset, mdt_count max_bytes,
                                mdt_count *actual);
/* Tuning knobs of the persistent launch.  policy: 0 = static strided split
 * of tiles over workgroups, 1 = dynamic (atomic tile counter), 2 = one tile
 * per workgroup run by a kernel without the tile loop (fewer scalar
 * registers held across the tile; requires wgs_per_cu = 0), 3 = each request
 * runs its single-request kernel (one launch, or graph node, per request;
 * requires wgs_per_cu = 0 and order = 0; a batch of one large request then
 * runs exactly as a plain launch).  order: 1 =
 * tiles run in the order of the typed address they start at, so requests
 * that touch the same memory (faces sharing cache lines) run together;
 * with policies 0 and 2 the ordered tiles are dealt to the XCDs (each has
 * its own L2) in groups of neighbours.  Other values: MDT_ERR_ARG. */
typedef struct mdt_batch_config {
    int tile_chunks;    /* 16-byte chunks per workgroup tile: 256, 512, 1024, 2048, 4096 */
    int wgs_per_cu;     /* persistent workgroups per compute unit, 1..16; 0: one workgroup per tile */
    int policy;         /* 0 static, 1 dynamic, 2 one tile per workgroup (no loop), 3 per-request kernels */
    int use_graph;      /* 1 = capture and replay a HIP graph, 0 = direct launches */
    int order;          /* 0 request order, 1 typed-address order */
} mdt_batch_config;
MDT_API int mdt_batch_set_config(mdt_batch b, const mdt_batch_config *cfg);
MDT_API int mdt_batch_get_config(mdt_batch b, mdt_batch_config *cfg);
/* Time candidate configurations on the batch as it stands -- tile size,
 * workgroups per CU, split policy, tile order, and graph replay against
 * direct launches -- running it several times (destinations are
 * overwritten with the same bytes), and keep the fastest.  *best may be
 * NULL. */
MDT_API int mdt_batch_autotune(mdt_batch b, mdt_stream s, mdt_batch_config *best);
/* Tune n batches of the same shape together (say the copies of a buffer a
 * caller rotates through, so every candidate is timed on inputs as they
 * run, out of cache): each candidate runs all n in turn, five times after
 * a warm-up, the median decides, and all n take the winner.  mdt_batch_autotune
 * is the n = 1 case.  With the environment variable MDT_AUTOTUNE_CACHE
 * naming a file, the choice is stored there under the batch's shape (per
 * request: direction, tile body, layout kind, type size, runs per element
 * and packed bytes to a power of two; the device's compute units; the
 * library version), and a later tuning of the same shape reads it back
 * instead of timing.  The file is a JSON object, one entry per line; it is
 * rewritten through a temporary file and a rename. */
MDT_API int mdt_batch_autotune_set(int n, mdt_batch *batches, mdt_stream s, mdt_batch_config *best);
MDT_API int mdt_batch_launch(mdt_batch b, mdt_stream s, mdt_request *req);
/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): as mdt_batch_launch,
 * but the batch's descriptors, tile prefix and tile counters live in a
 * fixed device array of the library (128 KiB, one per device, held until
 * the process ends) instead of the batch's own device buffers, and the call
 * allocates nothing: no device or host memory, no upload of type tables
 * (they are resident from the mdt_batch_add_* calls on this device; else
 * MDT_ERR_STATE).  Descriptors reach the array through small staging
 * kernels on stream s, followed by the batch kernels.  At most 1024
 * requests (MDT_ERR_NO_MEM beyond).  The batch's configuration applies,
 * except that tiles always run in request order (order = 1 is ignored).
 * The array is shared by every call on the device and keeps the last
 * call's contents: calls that overlap on one device (on different streams,
 * or from several threads without ordering) race; calls on one stream are
 * ordered.  Returns no request: completion is the stream's (record an
 * event after it). */
MDT_API int mdt_batch_launch_noalloc(mdt_batch b, mdt_stream s);

/* ---------------------------------------------------------------------
 * Serving: a progress engine that continuously batches pack/unpack
 * requests as they arrive, admits them against a device-memory budget and
 * runs them on its own HIP streams (General Progress: explicit progress or
 * a progress thread). */
typedef struct mdt_server_config {
    int nstreams;              /* HIP streams the server owns (default 8) */
    mdt_count budget_bytes;    /* admission budget (default 32 GiB) */
    int max_batch;             /* requests per launch (default 256) */
    int max_inflight;          /* launches in flight per stream (default 2) */
    mdt_count arena_bytes;     /* device arena for packed outputs; 0 = budget_bytes */
} mdt_server_config;
typedef struct mdt_server_stats {
    mdt_count submitted, completed, failed, deferred; /* deferred: admissions that waited */
    mdt_count bytes;           /* packed bytes moved by completed requests */
    mdt_count launches;        /* batched kernel launches */
    double p50_us, p99_us, max_us; /* latency: completion seen by host - submission */
    double elapsed_s;          /* first submission to last completion */
    mdt_count inflight_bytes, peak_inflight_bytes;
    double p50_queue_us, p99_queue_us; /* submission -> launch */
    double p50_run_us, p99_run_us;     /* launch -> completion seen by the progress engine */
    mdt_count direct;          /* requests launched by their own submit (nothing queued, a slot free) */
} mdt_server_stats;
MDT_API int mdt_server_create(const mdt_server_config *cfg, mdt_server *out);
/* Drains every admitted request, stops the progress thread, frees the
 * server. */
MDT_API int mdt_server_free(mdt_server *srv);
/* Submit a pack: bytes [inoffset, inoffset + actual) of (incount x t) at
 * inbuf into a packed buffer the server allocates from its arena; the
 * buffer is reported by mdt_server_request_result and released with the
 * request.  The type must stay valid until the request completes. */
MDT_API int mdt_server_submit_pack(mdt_server srv, const void *inbuf, mdt_count incount, mdt_type t,
                                   mdt_count inoffset, mdt_count max_pack_bytes, mdt_request *req);
/* Submit an unpack of the insize bytes at inbuf into (outcount x t) at
 * outbuf from stream position outoffset. */
MDT_API int mdt_server_submit_unpack(mdt_server srv, const void *inbuf, mdt_count insize, void *outbuf,
                                     mdt_count outcount, mdt_type t, mdt_count outoffset, mdt_request *req);
/* Server requests: poll with mdt_server_request_test (non-blocking; runs
 * progress when no progress thread is active), then read the result and
 * release the request (which returns its arena memory). */
MDT_API int mdt_server_request_test(mdt_server srv, mdt_request req, int *flag);
MDT_API int mdt_server_request_wait(mdt_server srv, mdt_request req);
/* *status: MDT_SUCCESS or the request's error; *packed: the device address
 * of the packed bytes (pack requests, else NULL); *nbytes: packed bytes;
 * *latency_us: completion minus submission. */
MDT_API int mdt_server_request_result(mdt_server srv, mdt_request req, int *status, void **packed,
                                      mdt_count *nbytes, double *latency_us);
MDT_API int mdt_server_request_release(mdt_server srv, mdt_request *req);
/* One round of progress: admit, launch, reap completions (MPIX_Stream_progress). */
MDT_API int mdt_server_progress(mdt_server srv);
MDT_API int mdt_server_start_progress_thread(mdt_server srv);
MDT_API int mdt_server_stop_progress_thread(mdt_server srv);
MDT_API int mdt_server_stats_get(mdt_server srv, mdt_server_stats *out);
/* Testing hook: make the next n arena allocations fail (MDT_ERR_NO_MEM is
 * then reported on those requests only). */
MDT_API int mdt_server_inject_alloc_failures(mdt_server srv, int n);

/* ---------------------------------------------------------------------
 * Diagnostics */
MDT_API const char *mdt_error_string(int code);
/* The last HIP error code seen by this thread (0 if none). */
MDT_API int mdt_last_hip_error(void);
/* Library version as 10000*major + 100*minor + patch. */
MDT_API int mdt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MDT_H */
