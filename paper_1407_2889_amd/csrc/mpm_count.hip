// Per-pattern occurrence counts of an ordered match list.
//
// The per-thread counts of Section 4.2 (each terminal adds the number of
// patterns it stands for) summed per pattern: counts[r] = number of pairs
// with id r. One pass over the list: every workgroup keeps a histogram of
// one slice of the id range in LDS, adds the pairs of its share of the list
// with LDS atomics, and flushes its nonzero bins to the global counts with
// one device atomic each. When the id range is wider than one LDS histogram
// the grid's second dimension walks the slices, so the list is read once per
// slice (a few slices at most: 40,960 bins per slice).

#include <hip/hip_runtime.h>

#include <algorithm>

#include "mpm_internal.h"

namespace mpm {
namespace {

constexpr uint32_t CNT_THREADS = 1024;
// Pairs each workgroup takes per pass of its grid-stride loop (4 per lane).
constexpr uint32_t CNT_UNROLL = 4;

__global__ void count_zero_kernel(uint32_t *__restrict__ counts, uint32_t d)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < d; i += stride)
        counts[i] = 0;
}

__device__ __forceinline__ void bin_add(uint32_t *bins, uint32_t id, uint32_t lo, uint32_t width)
{
    const uint32_t b = id - lo;  // ids below lo wrap to large values
    if (b < width)
        atomicAdd(&bins[b], 1u);
}

// blockIdx.y selects the id slice [lo, lo + width); the pairs are read with
// 8-byte loads (one pair per lane per load), CNT_UNROLL loads in flight.
__global__ __launch_bounds__(CNT_THREADS) void count_ids_kernel(
    const uint2 *__restrict__ pairs, uint64_t M, uint32_t d, uint32_t bins_per_slice,
    uint32_t *__restrict__ counts)
{
    extern __shared__ uint32_t bins[];
    const uint32_t lo = blockIdx.y * bins_per_slice;
    if (lo >= d)
        return;  // uniform over the workgroup
    const uint32_t width = min(bins_per_slice, d - lo);
    for (uint32_t b = threadIdx.x; b < width; b += CNT_THREADS)
        bins[b] = 0;
    __syncthreads();

    const uint64_t stride = (uint64_t)gridDim.x * CNT_THREADS;
    uint64_t i = (uint64_t)blockIdx.x * CNT_THREADS + threadIdx.x;
    for (; i + (CNT_UNROLL - 1) * stride < M; i += CNT_UNROLL * stride) {
        uint32_t id[CNT_UNROLL];
#pragma unroll
        for (uint32_t k = 0; k < CNT_UNROLL; ++k)
            id[k] = __builtin_nontemporal_load(&pairs[i + k * stride].y);
#pragma unroll
        for (uint32_t k = 0; k < CNT_UNROLL; ++k)
            bin_add(bins, id[k], lo, width);
    }
    for (; i < M; i += stride)
        bin_add(bins, __builtin_nontemporal_load(&pairs[i].y), lo, width);
    __syncthreads();

    for (uint32_t b = threadIdx.x; b < width; b += CNT_THREADS) {
        const uint32_t c = bins[b];
        if (c)
            atomicAdd(&counts[lo + b], c);
    }
}

}  // namespace
}  // namespace mpm

extern "C" mpm_status mpm_count_ids(const mpm_match *d_pairs, uint64_t M, uint32_t d,
                                    uint32_t *d_counts, void *stream)
{
    using namespace mpm;
    if (d == 0 || !d_counts || (M && !d_pairs) || (((uintptr_t)d_pairs) & 7u))
        return fail(MPM_EINVAL, "mpm_count_ids: bad arguments");
    int dev = 0, cus = 0, max_lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess)
        return fail(MPM_EHIP, "mpm_count_ids: %s", hipGetErrorString(e));
    if (cus <= 0 || max_lds < 4096)
        return fail(MPM_EHIP, "mpm_count_ids: device reports %d CUs, %d LDS bytes", cus, max_lds);
    hipStream_t s = (hipStream_t)stream;
    const uint32_t zero_grid = std::min<uint32_t>((d + 255) / 256, 1024);
    hipLaunchKernelGGL(count_zero_kernel, dim3(zero_grid), dim3(256), 0, s, d_counts, d);
    if (M) {
        // Balanced slices of at most max_lds / 4 bins.
        const uint32_t cap = (uint32_t)max_lds / 4;
        const uint32_t slices = (d + cap - 1) / cap;
        const uint32_t bins = ((d + slices - 1) / slices + 63) & ~63u;
        const uint32_t lds = bins * 4;
        const uint32_t per_cu = std::max<uint32_t>(1, std::min<uint32_t>(2, (uint32_t)max_lds / lds));
        // Enough pairs per workgroup that the flush (one atomic per nonzero
        // bin) stays small beside the pass over the list.
        const uint64_t want = (M + 65535) / 65536;
        const uint32_t gx = (uint32_t)std::max<uint64_t>(
            1, std::min<uint64_t>(want, (uint64_t)cus * per_cu / slices + 1));
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)count_ids_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(count_ids_kernel, dim3(gx, slices), dim3(CNT_THREADS), lds, s,
                           (const uint2 *)d_pairs, M, d, bins, d_counts);
    }
    e = hipGetLastError();
    if (e != hipSuccess)
        return fail(MPM_EHIP, "mpm_count_ids: %s", hipGetErrorString(e));
    return MPM_OK;
}
