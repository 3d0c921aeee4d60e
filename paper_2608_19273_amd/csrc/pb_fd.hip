// pb_fd.hip -- FD4 + KO6 + RK4 stage kernels (placeholder until implemented)
#include "pb_common.h"

namespace pb {

pb_status launch_fd_stage(pb_batch *, int, int, const void *, const void *, void *, void *, int, double,
                          double, hipStream_t)
{
    set_error("fd_ko_step: not implemented in this build");
    return PB_EUNSUPPORTED;
}

pb_status launch_fd_lambda(pb_batch *, double, hipStream_t)
{
    set_error("fd_ko_step: not implemented in this build");
    return PB_EUNSUPPORTED;
}

}  // namespace pb
