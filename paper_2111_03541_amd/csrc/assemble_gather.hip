// Owner-computes gather assembly for structured grids (placeholder until the kernel lands).
#include "mf_internal.h"

namespace mf {
mf_status assemble_gather(const AssembleArgs&) { return MF_ERR_UNSUPPORTED; }
}  // namespace mf
