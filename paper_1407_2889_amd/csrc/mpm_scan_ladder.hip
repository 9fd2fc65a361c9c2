// Scan kernels of the text-access ladder: Aho-Corasick reading its text a
// byte at a time from global memory, or from a copy staged in LDS.
#include "mpm_scan_impl.h"

namespace mpm {

template <int TM>
static const void *ladder_pick(const LaunchCfg &c)
{
    return c.placement == MPM_PLACE_LDS ? pick_w<AcTextWalk<uint16_t, PL_LDS, TM>>(c.block_threads)
                                        : pick_w<AcTextWalk<uint16_t, PL_GLB, TM>>(c.block_threads);
}

const void *ladder_kernel(const mpm_index * /*ix*/, const LaunchCfg &c)
{
    return c.text_mode == 1 ? ladder_pick<1>(c) : ladder_pick<2>(c);
}

template <int TM>
static hipError_t ladder_go(const AcDev &a, const LaunchCfg &c, const ScanDev &sd, hipStream_t s)
{
    if (c.placement == MPM_PLACE_LDS)
        return launch_w<AcTextWalk<uint16_t, PL_LDS, TM>>(a, c, sd, a.uoff, a.uids, a.dupfree,
                                                          c.text_lds, s);
    return launch_w<AcTextWalk<uint16_t, PL_GLB, TM>>(a, c, sd, a.uoff, a.uids, a.dupfree,
                                                      c.text_lds, s);
}

mpm_status ladder_launch(const mpm_index *ix, const LaunchCfg &c, const ScanDev &sd, void *stream)
{
    const AcDev a = ac_dev(ix);
    const hipError_t e = c.text_mode == 1 ? ladder_go<1>(a, c, sd, (hipStream_t)stream)
                                          : ladder_go<2>(a, c, sd, (hipStream_t)stream);
    if (e != hipSuccess)
        return fail(MPM_EHIP, "scan launch: %s", hipGetErrorString(e));
    return MPM_OK;
}

}  // namespace mpm
