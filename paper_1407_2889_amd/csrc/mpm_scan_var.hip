// Scan kernels for pattern sets of different lengths: Aho-Corasick over the
// reversed strings and Wu-Manber on the shortest length (LDS, hot rows in
// LDS, or global memory).
#include "mpm_scan_impl.h"

namespace mpm {

const void *var_kernel(const mpm_index *ix, const LaunchCfg &c)
{
    const uint32_t W = c.block_threads;
    if (ix->algo == MPM_ALGO_AC) {
        if (ix->state_bytes == 4)
            return c.placement == MPM_PLACE_HOT ? pick_w<AcRevWalk<uint32_t, PL_HOT>>(W)
                                                : pick_w<AcRevWalk<uint32_t, PL_GLB>>(W);
        return c.placement == MPM_PLACE_LDS   ? pick_w<AcRevWalk<uint16_t, PL_LDS>>(W)
               : c.placement == MPM_PLACE_HOT ? pick_w<AcRevWalk<uint16_t, PL_HOT>>(W)
                                              : pick_w<AcRevWalk<uint16_t, PL_GLB>>(W);
    }
    if (c.placement == MPM_PLACE_HOT)
        return pick_w<WmWalk<PL_HOT, true>>(W);
    return c.placement == MPM_PLACE_LDS ? pick_w<WmWalk<PL_LDS, true>>(W)
                                        : pick_w<WmWalk<PL_GLB, true>>(W);
}

mpm_status var_launch(const mpm_index *ix, const LaunchCfg &c, const ScanDev &sd, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (ix->algo == MPM_ALGO_AC) {
        const AcDev a = ac_dev(ix);
        if (ix->state_bytes == 4 && c.placement == MPM_PLACE_HOT)
            e = launch_w<AcRevWalk<uint32_t, PL_HOT>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
        else if (ix->state_bytes == 4)
            e = launch_w<AcRevWalk<uint32_t, PL_GLB>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
        else if (c.placement == MPM_PLACE_HOT)
            e = launch_w<AcRevWalk<uint16_t, PL_HOT>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
        else if (c.placement == MPM_PLACE_LDS)
            e = launch_w<AcRevWalk<uint16_t, PL_LDS>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
        else
            e = launch_w<AcRevWalk<uint16_t, PL_GLB>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
    } else {
        const WmDev a = wm_dev(ix);
        if (c.placement == MPM_PLACE_HOT)
            e = launch_w<WmWalk<PL_HOT, true>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
        else if (c.placement == MPM_PLACE_LDS)
            e = launch_w<WmWalk<PL_LDS, true>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
        else
            e = launch_w<WmWalk<PL_GLB, true>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
    }
    if (e != hipSuccess)
        return fail(MPM_EHIP, "scan launch: %s", hipGetErrorString(e));
    return MPM_OK;
}

}  // namespace mpm
