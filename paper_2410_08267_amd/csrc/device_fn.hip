// The device's own evaluation of elementary functions of the right-hand side
// (the NFW mass integral, the power-law factors of K and Kc), one value per
// thread, for tests of their accuracy: the same inline code the trajectory
// kernels run.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "nh_device.h"
#include "nh_launch.h"

namespace nh {

__global__ __launch_bounds__(256) void k_device_fn(int fn, PowFactor pw, long long n, const double *x, double *y)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        y[i] = fn == FN_NFW_I ? nfw_I(x[i]) : pow_factor(pw, x[i]);
}

hipError_t launch_device_fn(int fn, const PowFactor &pw, long long n, const double *x, double *y, hipStream_t s)
{
    const long long blocks = std::min<long long>((n + 255) / 256, 4096);
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_device_fn, dim3((unsigned)blocks), dim3(256), 0, s, fn, pw, n, x, y);
    return hipGetLastError();
}

}  // namespace nh
