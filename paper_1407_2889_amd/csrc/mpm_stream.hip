// Scanning a text that stays in host memory.
//
// The paper's texts were larger than device memory and were read by the
// kernels straight from host memory (Section 5). Here the text is cut into
// chunks of starting positions; each chunk, with the m - 1 bytes that follow
// it, is copied into one of two device staging buffers on a copy stream
// while the previous chunk is scanned, so the link stays busy. A chunk
// reports exactly the starting positions it owns (its last window ends at its
// last byte), the pairs go to the output after those of earlier chunks, and a
// small kernel adds the chunk's offset in the text to their positions.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "mpm_internal.h"

namespace mpm {
namespace {

// pairs: (pos, id) words; adds base to every pos.
__global__ void add_base_kernel(uint32_t *__restrict__ pairs, uint64_t count, uint32_t base)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        pairs[2 * i] += base;
}

// Copy stream and events of one call, released on every exit path.
struct StreamSet {
    hipStream_t copy = nullptr;
    hipEvent_t ready[2] = {nullptr, nullptr};
    ~StreamSet()
    {
        if (copy) {
            (void)hipStreamSynchronize(copy);
            (void)hipStreamDestroy(copy);
        }
        for (hipEvent_t e : ready)
            if (e)
                (void)hipEventDestroy(e);
    }
};

}  // namespace
}  // namespace mpm

extern "C" mpm_status mpm_scan_host(const mpm_index *idx, const uint8_t *h_text, uint64_t n,
                                    uint8_t *d_stage, uint64_t stage_bytes, uint64_t chunk,
                                    mpm_match *d_out,
                                    uint64_t capacity, void *d_work, uint64_t work_bytes,
                                    uint64_t *d_total, const mpm_variant *v, void *stream,
                                    uint64_t *total)
{
    using namespace mpm;
    if (!idx || !total || !d_total || !d_work || !d_stage || chunk == 0 || (n && !h_text) ||
        (capacity && !d_out))
        return fail(MPM_EINVAL, "mpm_scan_host: null argument or zero chunk");
    if (idx->var)
        return fail(MPM_EUNSUPPORTED, "mpm_scan_host: sets of different lengths need the whole "
                    "text on the device");
    if (n >= (1ull << 32))
        return fail(MPM_ETOOBIG, "mpm_scan_host: n = %llu needs 32-bit positions",
                    (unsigned long long)n);
    const uint32_t m = idx->m;
    if (chunk > (1ull << 32) - m)
        return fail(MPM_EINVAL, "mpm_scan_host: chunk of %llu positions is too large",
                    (unsigned long long)chunk);
    hipStream_t s = (hipStream_t)stream;
    *total = 0;
    const uint64_t ns = n >= m ? n - m + 1 : 0;
    if (ns == 0)
        return mpm_scan_sync(idx, d_stage, 0, d_out, capacity, d_work, work_bytes, d_total, v,
                             stream, total);
    chunk = std::min(chunk, ns);
    const uint64_t nchunks = (ns + chunk - 1) / chunk;
    const uint64_t buf_bytes = chunk + m - 1;
    if (stage_bytes < (nchunks > 1 ? 2 : 1) * buf_bytes)
        return fail(MPM_ENOMEM, "mpm_scan_host: staging buffer of %llu bytes, need %llu",
                    (unsigned long long)stage_bytes,
                    (unsigned long long)((nchunks > 1 ? 2 : 1) * buf_bytes));
    StreamSet ss;
    if (hipStreamCreateWithFlags(&ss.copy, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ss.ready[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ss.ready[1], hipEventDisableTiming) != hipSuccess)
        return fail(MPM_EHIP, "mpm_scan_host: stream or event creation failed");
    // Byte range of chunk k: its starting positions and the m - 1 bytes after them.
    auto bytes_of = [&](uint64_t k) { return std::min(n, (k + 1) * chunk + m - 1) - k * chunk; };
    auto copy = [&](uint64_t k) -> hipError_t {
        uint8_t *dst = d_stage + (k & 1) * buf_bytes;
        hipError_t e = hipMemcpyAsync(dst, h_text + k * chunk, bytes_of(k),
                                      hipMemcpyHostToDevice, ss.copy);
        return e == hipSuccess ? hipEventRecord(ss.ready[k & 1], ss.copy) : e;
    };
    hipError_t e = copy(0);
    uint64_t written = 0;
    for (uint64_t k = 0; k < nchunks && e == hipSuccess; ++k) {
        // The other buffer was last read by the scan of chunk k - 1, which
        // the host has already waited for.
        if (k + 1 < nchunks && (e = copy(k + 1)) != hipSuccess)
            break;
        if ((e = hipStreamWaitEvent(s, ss.ready[k & 1], 0)) != hipSuccess)
            break;
        const uint64_t left = capacity > written ? capacity - written : 0;
        uint64_t tk = 0;
        mpm_status st = mpm_scan_sync(idx, d_stage + (k & 1) * buf_bytes, bytes_of(k),
                                      left ? d_out + written : nullptr, left, d_work, work_bytes,
                                      d_total, v, stream, &tk);
        if (st != MPM_OK && st != MPM_EOVERFLOW)
            return st;
        const uint64_t wrote = std::min(tk, left);
        if (wrote && k) {
            const uint32_t grid = (uint32_t)std::min<uint64_t>((wrote + 255) / 256, 8192);
            hipLaunchKernelGGL(add_base_kernel, dim3(grid), dim3(256), 0, s,
                               (uint32_t *)(d_out + written), wrote, (uint32_t)(k * chunk));
            e = hipGetLastError();
        }
        written += tk;
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail(MPM_EHIP, "mpm_scan_host: %s", hipGetErrorString(e));
    *total = written;
    if (written > capacity)
        return fail(MPM_EOVERFLOW, "mpm_scan_host: %llu matches, capacity %llu",
                    (unsigned long long)written, (unsigned long long)capacity);
    return MPM_OK;
}
