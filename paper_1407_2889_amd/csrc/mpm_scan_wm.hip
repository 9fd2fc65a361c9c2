// Wu-Manber scan kernels.
#include "mpm_scan_impl.h"

namespace mpm {

const void *wm_kernel(const LaunchCfg &c)
{
    return c.placement == MPM_PLACE_LDS ? pick_w<WmWalk<true>>(c.block_threads)
                                        : pick_w<WmWalk<false>>(c.block_threads);
}

hipError_t wm_launch(const WmDev &a, const LaunchCfg &c, const ScanDev &sd, hipStream_t s)
{
    return c.placement == MPM_PLACE_LDS ? launch_w<WmWalk<true>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s)
                                        : launch_w<WmWalk<false>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
}

}  // namespace mpm
