// batch_p1u0.hip -- batch kernel variants for the dynamic split, pack (and copy) direction.
#include "batch_kernel.h"

namespace mdt {

template <>
void launch_batch_dir<1, 0>(dim3 grid, size_t lds, hipStream_t s, const BatchHeader *H, const ReqDesc *R,
                            const int64_t *tile0, const int32_t *order, unsigned long long *counter, int body)
{
    launch_batch_dir_impl<1, 0>(grid, lds, s, H, R, tile0, order, counter, body);
}

}  // namespace mdt
