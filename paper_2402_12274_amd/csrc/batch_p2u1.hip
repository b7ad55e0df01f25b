// batch_p2u1.hip -- batch kernel variants for one tile per workgroup, unpack direction.
#include "batch_kernel.h"

namespace mdt {

template <>
void launch_batch_dir<2, 1>(dim3 grid, size_t lds, hipStream_t s, const BatchHeader *H, const ReqDesc *R,
                            const int64_t *tile0, const int32_t *order, unsigned long long *counter, int body)
{
    launch_batch_dir_impl<2, 1>(grid, lds, s, H, R, tile0, order, counter, body);
}

}  // namespace mdt
