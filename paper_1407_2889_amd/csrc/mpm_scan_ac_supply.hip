// Aho-Corasick scan kernels walking the goto function and supply links
// (the paper's kernel design, kept beside the flattened walk for comparison):
// uint16_t or uint32_t entries, tables in LDS or global memory.
#include "mpm_scan_impl.h"

namespace mpm {

const void *ac_supply_kernel(uint32_t state_bytes, const LaunchCfg &c)
{
    const bool lds = c.placement == MPM_PLACE_LDS;
    if (state_bytes == 2)
        return lds ? pick_w<AcSupplyWalk<uint16_t, PL_LDS>>(c.block_threads)
                   : pick_w<AcSupplyWalk<uint16_t, PL_GLB>>(c.block_threads);
    return lds ? pick_w<AcSupplyWalk<uint32_t, PL_LDS>>(c.block_threads)
               : pick_w<AcSupplyWalk<uint32_t, PL_GLB>>(c.block_threads);
}

hipError_t ac_supply_launch(uint32_t state_bytes, const AcDev &a, const LaunchCfg &c,
                            const ScanDev &sd, hipStream_t s)
{
    const bool lds = c.placement == MPM_PLACE_LDS;
    if (state_bytes == 2)
        return lds ? launch_w<AcSupplyWalk<uint16_t, PL_LDS>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s)
                   : launch_w<AcSupplyWalk<uint16_t, PL_GLB>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
    return lds ? launch_w<AcSupplyWalk<uint32_t, PL_LDS>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s)
               : launch_w<AcSupplyWalk<uint32_t, PL_GLB>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
}

}  // namespace mpm
