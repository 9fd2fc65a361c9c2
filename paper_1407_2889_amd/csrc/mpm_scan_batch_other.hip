// Batched persistent kernels: Aho-Corasick with 32-bit table entries (global
// or hot placement) and
// Wu-Manber (one kernel per table placement, byte-class method and block size).
#include "mpm_scan_impl.h"

namespace mpm {

const void *batch_kernel_other(uint32_t kind, uint32_t W)
{
    const bool swar = (kind & BK_SWAR) != 0;
    switch (kind & BK_WALK_MASK) {
    case BK_AC32_GLB:
        return swar ? batch_pick_w<AcWalk<uint32_t, PL_GLB, true, 1>>(W)
                    : batch_pick_w<AcWalk<uint32_t, PL_GLB, false, 1>>(W);
    case BK_AC32_HOT:
        return swar ? batch_pick_w<AcWalk<uint32_t, PL_HOT, true, 1>>(W)
                    : batch_pick_w<AcWalk<uint32_t, PL_HOT, false, 1>>(W);
    case BK_WM_LDS: return batch_pick_w<WmWalk<PL_LDS>>(W);
    case BK_WM_HOT: return batch_pick_w<WmWalk<PL_HOT>>(W);
    case BK_WM_GLB: return batch_pick_w<WmWalk<PL_GLB>>(W);
    }
    return nullptr;
}

hipError_t batch_launch_other(const BatchDev &bd, uint32_t kind, uint32_t W, uint32_t grid,
                              uint32_t lds, hipStream_t s)
{
    const bool swar = (kind & BK_SWAR) != 0;
    switch (kind & BK_WALK_MASK) {
    case BK_AC32_GLB:
        return swar ? batch_launch_w<AcWalk<uint32_t, PL_GLB, true, 1>>(bd, W, grid, lds, s)
                    : batch_launch_w<AcWalk<uint32_t, PL_GLB, false, 1>>(bd, W, grid, lds, s);
    case BK_AC32_HOT:
        return swar ? batch_launch_w<AcWalk<uint32_t, PL_HOT, true, 1>>(bd, W, grid, lds, s)
                    : batch_launch_w<AcWalk<uint32_t, PL_HOT, false, 1>>(bd, W, grid, lds, s);
    case BK_WM_LDS: return batch_launch_w<WmWalk<PL_LDS>>(bd, W, grid, lds, s);
    case BK_WM_HOT: return batch_launch_w<WmWalk<PL_HOT>>(bd, W, grid, lds, s);
    case BK_WM_GLB: return batch_launch_w<WmWalk<PL_GLB>>(bd, W, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace mpm
