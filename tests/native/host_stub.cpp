// host_stub.cpp -- the device side of the layout compiler replaced for
// host-only builds (types.cpp and compile.cpp compiled unchanged with the
// host compiler, under AddressSanitizer and UndefinedBehaviorSanitizer):
// there is no device, so commit keeps its tables on the host, as it does on
// a machine without a GPU.
#include "core.h"

namespace mdt {

int device_tables(Compiled *, DeviceTables **out)
{
    *out = nullptr;
    return MDT_ERR_HIP;  // no device: commit proceeds without resident tables
}

void free_device_tables(DeviceTables *) {}

}  // namespace mdt
