// Measurement kernel (not part of the matching method): the HBM read rate of
// the scan's text access pattern without its table walk. Every lane of a
// 1024-thread workgroup reads its own lane_bytes range as whole 128-byte
// lines (eight 16-byte loads issued together, the next line in flight while
// the current one is folded), the ranges of a workgroup's lanes side by side
// and one chunk of 1024 ranges per workgroup, as the scans lay out one
// chunk per workgroup.
#include <hip/hip_runtime.h>

#include "mpm_internal.h"

namespace mpm {
namespace {

typedef uint32_t pv4u __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(1024) void read_lanes_kernel(const pv4u *__restrict__ p,
                                                          uint32_t lane_lines, uint32_t sentinel,
                                                          uint32_t *sink)
{
    const uint64_t lane = (uint64_t)blockIdx.x * 1024 + threadIdx.x;
    const pv4u *q = p + lane * lane_lines * 8;
    uint32_t acc = 0;
    pv4u c[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
        c[j] = q[j];
    for (uint32_t l = 0; l < lane_lines; ++l) {
        const uint32_t nl = l + 1 < lane_lines ? l + 1 : l;
        pv4u nx[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            nx[j] = q[nl * 8 + j];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            acc += c[j].x ^ c[j].y ^ c[j].z ^ c[j].w;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            c[j] = nx[j];
    }
    if (acc == sentinel)
        sink[0] = acc;
}

}  // namespace
}  // namespace mpm

extern "C" mpm_status mpm_read_probe_lanes(const uint8_t *d_buf, uint64_t bytes,
                                           uint32_t lane_bytes, uint32_t *d_sink, void *stream)
{
    using namespace mpm;
    if (!d_buf || !d_sink || (((uintptr_t)d_buf) & 127u))
        return fail(MPM_EINVAL, "mpm_read_probe_lanes: null or unaligned buffer");
    if (lane_bytes == 0 || lane_bytes % 128 || bytes == 0 || bytes % (1024ull * lane_bytes))
        return fail(MPM_EINVAL, "mpm_read_probe_lanes: lane_bytes must be a positive multiple of "
                    "128 and bytes a multiple of 1024 lanes of it");
    const uint64_t grid = bytes / (1024ull * lane_bytes);
    if (grid > 0x7fffffffull)
        return fail(MPM_EINVAL, "mpm_read_probe_lanes: too many workgroups");
    hipLaunchKernelGGL(read_lanes_kernel, dim3((uint32_t)grid), dim3(1024), 0, (hipStream_t)stream,
                       (const pv4u *)d_buf, lane_bytes / 128, 0xA5C3E1F7u, d_sink);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(MPM_EHIP, "mpm_read_probe_lanes: %s", hipGetErrorString(e));
    return MPM_OK;
}
