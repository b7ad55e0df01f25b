/* Plain C99 client of include/mdt.h: compiles without HIP headers and
 * exercises the host-only calls (constructors, attributes, segment queries,
 * error codes).  Exit status 0 on success. */
#include <stdio.h>
#include <stdint.h>
#include <string.h>
#include <sys/uio.h>

#include "mdt.h"

#define CHECK(cond)                                                    \
    do {                                                               \
        if (!(cond)) {                                                 \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            return 1;                                                  \
        }                                                              \
    } while (0)

int main(void)
{
    /* mdt_iov is layout-compatible with struct iovec */
    CHECK(sizeof(mdt_iov) == sizeof(struct iovec));
    CHECK(offsetof(mdt_iov, iov_len) == offsetof(struct iovec, iov_len));

    mdt_type value, volume;
    CHECK(mdt_type_contiguous(16, MDT_BYTE, &value) == MDT_SUCCESS);
    mdt_count full[3] = {1000, 1000, 1000}, sub[3] = {100, 100, 100}, start[3] = {300, 300, 300};
    CHECK(mdt_type_create_subarray(3, full, sub, start, MDT_ORDER_C, value, &volume) == MDT_SUCCESS);
    mdt_count n, bytes;
    CHECK(mdt_type_iov_len(volume, -1, &n, &bytes) == MDT_ERR_TYPE); /* not committed */
    CHECK(mdt_type_commit(&volume) == MDT_SUCCESS);
    CHECK(mdt_type_iov_len(volume, 2147483647, &n, &bytes) == MDT_SUCCESS);
    CHECK(n == 10000 && bytes == 16000000);
    mdt_iov iov[4];
    mdt_count got;
    CHECK(mdt_type_iov(volume, 0, iov, 4, &got) == MDT_SUCCESS && got == 4);
    CHECK((intptr_t)iov[0].iov_base == 4804804800LL && iov[0].iov_len == 1600);
    CHECK((intptr_t)iov[3].iov_base == 4804852800LL);
    CHECK(mdt_type_iov_len(volume, -2, &n, &bytes) == MDT_ERR_ARG);
    mdt_aint lb, ext;
    CHECK(mdt_type_get_extent(volume, &lb, &ext) == MDT_SUCCESS && lb == 0 && ext == 16000000000LL);
    /* errors leave outputs untouched */
    mdt_type bad = (mdt_type)0x1;
    mdt_type out = MDT_TYPE_NULL;
    mdt_count sz = -7;
    CHECK(mdt_type_size(MDT_TYPE_NULL, &sz) == MDT_ERR_TYPE && sz == -7);
    CHECK(mdt_type_vector(-1, 1, 1, MDT_DOUBLE, &out) == MDT_ERR_ARG && out == MDT_TYPE_NULL);
    CHECK(mdt_type_contiguous(1, MDT_TYPE_NULL, &out) == MDT_ERR_TYPE);
    (void)bad;
    CHECK(mdt_type_free(&volume) == MDT_SUCCESS && volume == MDT_TYPE_NULL);
    CHECK(mdt_type_free(&value) == MDT_SUCCESS);
    mdt_type dbl = MDT_DOUBLE;
    CHECK(mdt_type_free(&dbl) == MDT_ERR_TYPE); /* predefined types are not freed */
    CHECK(strlen(mdt_error_string(MDT_ERR_OVERLAP)) > 0);
    CHECK(mdt_version() >= 100);
    printf("abi ok\n");
    return 0;
}
