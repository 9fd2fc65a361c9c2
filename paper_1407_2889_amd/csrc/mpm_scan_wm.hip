// Wu-Manber scan kernels.
#include "mpm_scan_impl.h"

namespace mpm {

const void *wm_kernel(const LaunchCfg &c)
{
    if (c.dense)
        return c.placement == MPM_PLACE_HOT   ? pick_dense<WmWalk<PL_HOT>>()
               : c.placement == MPM_PLACE_LDS ? pick_dense<WmWalk<PL_LDS>>()
                                              : pick_dense<WmWalk<PL_GLB>>();
    if (c.placement == MPM_PLACE_HOT)
        return pick_w<WmWalk<PL_HOT>>(c.block_threads);
    return c.placement == MPM_PLACE_LDS ? pick_w<WmWalk<PL_LDS>>(c.block_threads)
                                        : pick_w<WmWalk<PL_GLB>>(c.block_threads);
}

hipError_t wm_launch(const WmDev &a, const LaunchCfg &c, const ScanDev &sd, hipStream_t s)
{
    if (c.dense)
        return c.placement == MPM_PLACE_HOT   ? launch_dense<WmWalk<PL_HOT>>(a, c, sd, a.uoff, a.uids, a.dupfree, s)
               : c.placement == MPM_PLACE_LDS ? launch_dense<WmWalk<PL_LDS>>(a, c, sd, a.uoff, a.uids, a.dupfree, s)
                                              : launch_dense<WmWalk<PL_GLB>>(a, c, sd, a.uoff, a.uids, a.dupfree, s);
    if (c.placement == MPM_PLACE_HOT)
        return launch_w<WmWalk<PL_HOT>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
    return c.placement == MPM_PLACE_LDS ? launch_w<WmWalk<PL_LDS>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s)
                                        : launch_w<WmWalk<PL_GLB>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
}

}  // namespace mpm
