// FP32-compensated Dormand-Prince kernel (placeholder until the FP32C path lands).
#include <hip/hip_runtime.h>

#include "nh_device.h"

namespace nh {

hipError_t launch_dp5_f32c(const TrajParams &P, const GridPtrs &g, const TrajOut &o,
                           unsigned long long *counter, int n_cu, hipStream_t s)
{
    (void)P; (void)g; (void)o; (void)counter; (void)n_cu; (void)s;
    return hipErrorNotSupported;
}

}  // namespace nh
