// Aho-Corasick scan kernels: uint16_t table entries, table in LDS.
#include "mpm_scan_impl.h"

namespace mpm {

const void *ac16_lds_kernel(const LaunchCfg &c)
{
    const bool sw = c.swar, i2 = c.ilp == 2;
    if (c.dense)
        return sw ? pick_dense<AcWalk<uint16_t, true, true, 1>>()
                  : pick_dense<AcWalk<uint16_t, true, false, 1>>();
    return sw ? (i2 ? pick_w<AcWalk<uint16_t, true, true, 2>>(c.block_threads)
                    : pick_w<AcWalk<uint16_t, true, true, 1>>(c.block_threads))
              : (i2 ? pick_w<AcWalk<uint16_t, true, false, 2>>(c.block_threads)
                    : pick_w<AcWalk<uint16_t, true, false, 1>>(c.block_threads));
}

hipError_t ac16_lds_launch(const AcDev &a, const LaunchCfg &c, const ScanDev &sd, hipStream_t s)
{
    const bool sw = c.swar, i2 = c.ilp == 2;
    if (c.dense)
        return sw ? launch_dense<AcWalk<uint16_t, true, true, 1>>(a, c, sd, a.uoff, a.uids, a.dupfree, s)
                  : launch_dense<AcWalk<uint16_t, true, false, 1>>(a, c, sd, a.uoff, a.uids, a.dupfree, s);
    if (sw)
        return i2 ? launch_w<AcWalk<uint16_t, true, true, 2>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s)
                  : launch_w<AcWalk<uint16_t, true, true, 1>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
    return i2 ? launch_w<AcWalk<uint16_t, true, false, 2>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s)
              : launch_w<AcWalk<uint16_t, true, false, 1>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
}

}  // namespace mpm
