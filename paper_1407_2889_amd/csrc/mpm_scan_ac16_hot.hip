// Aho-Corasick scan kernels: uint16_t table entries, the first rows (in
// breadth-first order) in LDS and the rest in global memory. One chain per
// lane.
#include "mpm_scan_impl.h"

namespace mpm {

const void *ac16_hot_kernel(const LaunchCfg &c)
{
    if (c.dense)
        return c.swar ? pick_dense<AcWalk<uint16_t, PL_HOT, true, 1>>()
                      : pick_dense<AcWalk<uint16_t, PL_HOT, false, 1>>();
    return c.swar ? pick_w<AcWalk<uint16_t, PL_HOT, true, 1>>(c.block_threads)
                  : pick_w<AcWalk<uint16_t, PL_HOT, false, 1>>(c.block_threads);
}

hipError_t ac16_hot_launch(const AcDev &a, const LaunchCfg &c, const ScanDev &sd, hipStream_t s)
{
    if (c.dense)
        return c.swar ? launch_dense<AcWalk<uint16_t, PL_HOT, true, 1>>(a, c, sd, a.uoff, a.uids, a.dupfree, s)
                      : launch_dense<AcWalk<uint16_t, PL_HOT, false, 1>>(a, c, sd, a.uoff, a.uids, a.dupfree, s);
    return c.swar ? launch_w<AcWalk<uint16_t, PL_HOT, true, 1>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s)
                  : launch_w<AcWalk<uint16_t, PL_HOT, false, 1>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
}

}  // namespace mpm
