// Single-text scan on the library's own per-device scratch (mpm_scan_noalloc):
// the same launch as mpm_scan, with the workspace (ticket and done counters,
// launch epoch, error word, one look-back status word per chunk) taken from a
// file-scope device array instead of a caller buffer. Nothing here allocates.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>

#include "mpm_internal.h"

namespace mpm {
mpm_status workspace_sizes(const mpm_index *idx, uint64_t n, const mpm_variant *v,
                           uint64_t *min_bytes, uint64_t *full_bytes, const char *who);
mpm_status scan_with_workspace(const mpm_index *idx, const uint8_t *d_text, uint64_t n,
                               mpm_match *d_out, uint64_t capacity, void *d_work,
                               uint64_t work_bytes, uint64_t *d_total, const mpm_variant *v,
                               void *stream, const char *who);
}  // namespace mpm

// One copy per device, kept until the process ends. In host code this name is
// a host-side stand-in: kernels and copies get the device address that
// hipGetSymbolAddress returns for it (scratch_address below).
static __device__ __align__(256) uint8_t scratch[MPM_NOALLOC_SCRATCH_BYTES];

namespace {

// Zero the scratch once per device (a kernel, not a memset, so that a first
// call made under stream capture records a plain kernel node).
__global__ void zero_scratch_kernel(uint4 *p, uint64_t n16)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0, 0, 0, 0);
}

std::mutex g_mu;
const int MAX_DEVICES = 64;
void *g_ptr[MAX_DEVICES] = {nullptr};

// Device address of this device's scratch; on the first call for a device
// (with it current) looks the address up and enqueues the zero fill on
// `stream`, ahead of the scan that follows on the same stream.
mpm_status scratch_address(void *stream, void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return mpm::fail(MPM_EHIP, "mpm_scan_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES)
        return mpm::fail(MPM_EUNSUPPORTED, "mpm_scan_noalloc: device %d beyond %d", dev,
                         MAX_DEVICES);
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return mpm::fail(MPM_EHIP, "mpm_scan_noalloc: hipGetSymbolAddress: %s",
                             hipGetErrorString(e));
        hipLaunchKernelGGL(zero_scratch_kernel, dim3(64), dim3(256), 0, (hipStream_t)stream,
                           (uint4 *)p, (uint64_t)(MPM_NOALLOC_SCRATCH_BYTES / 16));
        e = hipGetLastError();
        if (e != hipSuccess)
            return mpm::fail(MPM_EHIP, "mpm_scan_noalloc: scratch fill: %s", hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return MPM_OK;
}

}  // namespace

extern "C" mpm_status mpm_scan_noalloc(const mpm_index *idx, const uint8_t *d_text, uint64_t n,
                                       mpm_match *d_out, uint64_t capacity, uint64_t *d_total,
                                       const mpm_variant *v, void *stream)
{
    using namespace mpm;
    if (!idx || !d_total)
        return fail(MPM_EINVAL, "mpm_scan_noalloc: null index or total");
    // the header and status words must fit; staging takes whatever is left
    uint64_t need = 0;
    mpm_status st = workspace_sizes(idx, n, v, &need, &need, "mpm_scan_noalloc");
    if (st)
        return st;
    if (need > MPM_NOALLOC_SCRATCH_BYTES)
        return fail(MPM_ENOMEM, "mpm_scan_noalloc: the scan needs %llu bytes of scratch, the "
                    "static scratch holds %llu (use larger lane_bytes or block_threads, or "
                    "mpm_scan with a workspace)", (unsigned long long)need,
                    (unsigned long long)MPM_NOALLOC_SCRATCH_BYTES);
    void *ptr = nullptr;
    st = scratch_address(stream, &ptr);
    if (st)
        return st;
    return scan_with_workspace(idx, d_text, n, d_out, capacity, ptr, MPM_NOALLOC_SCRATCH_BYTES,
                               d_total, v, stream, "mpm_scan_noalloc");
}
