// Learned preconditioner (placeholder until the network kernels land).
#include "mf_internal.h"
#include "pcg.h"

namespace mf {
mf_status nn_bind_pcg(const mf_nn_t*, int64_t, PcgArgs*)
{
    return set_error(MF_ERR_UNSUPPORTED, "learned preconditioner not built");
}
}  // namespace mf
