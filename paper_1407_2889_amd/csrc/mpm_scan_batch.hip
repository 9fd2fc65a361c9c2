// Batched persistent kernels (one per block size).
#include "mpm_scan_impl.h"

namespace mpm {

const void *batch_kernel_ptr(uint32_t W)
{
    switch (W) {
    case 256: return (const void *)batch_kernel<256>;
    case 512: return (const void *)batch_kernel<512>;
    case 1024: return (const void *)batch_kernel<1024>;
    }
    return nullptr;
}

hipError_t batch_launch(const BatchDev &bd, uint32_t W, uint32_t grid, uint32_t lds, hipStream_t s)
{
    switch (W) {
    case 256: hipLaunchKernelGGL(batch_kernel<256>, dim3(grid), dim3(256), lds, s, bd); break;
    case 512: hipLaunchKernelGGL(batch_kernel<512>, dim3(grid), dim3(512), lds, s, bd); break;
    default: hipLaunchKernelGGL(batch_kernel<1024>, dim3(grid), dim3(1024), lds, s, bd); break;
    }
    return hipGetLastError();
}

}  // namespace mpm
