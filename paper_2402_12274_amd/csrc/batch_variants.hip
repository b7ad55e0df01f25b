// batch_variants.hip -- the batch kernel variants of one launch policy and
// direction.  The build compiles this file once per (policy, direction) pair,
// with MDT_BATCH_POLICY (0 static split, 1 dynamic split, 2 one tile per
// workgroup) and MDT_BATCH_UNPACK (0 pack and copy, 1 unpack) defined, so the
// six sets of tile-body instantiations compile as separate translation units.
#include "batch_kernel.h"

#if !defined(MDT_BATCH_POLICY) || !defined(MDT_BATCH_UNPACK)
#error "compile with -DMDT_BATCH_POLICY=<0|1|2> -DMDT_BATCH_UNPACK=<0|1>"
#endif

namespace mdt {

template <>
void launch_batch_dir<MDT_BATCH_POLICY, MDT_BATCH_UNPACK>(dim3 grid, size_t lds, hipStream_t s, const BatchHeader *H,
                                                          const ReqDesc *R, const int64_t *tile0, const int32_t *order,
                                                          unsigned long long *counter, int body)
{
    launch_batch_dir_impl<MDT_BATCH_POLICY, MDT_BATCH_UNPACK>(grid, lds, s, H, R, tile0, order, counter, body);
}

}  // namespace mdt
