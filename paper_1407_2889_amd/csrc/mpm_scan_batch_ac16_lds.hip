// Batched persistent kernels: Aho-Corasick with 16-bit table entries,
// the table in LDS (both byte-class methods, every block size).
#include "mpm_scan_impl.h"

namespace mpm {

MPM_BATCH_AC16_TU(PL_LDS)

}  // namespace mpm
