// pb_srhd.hip -- SRHD con2prim pass (placeholder until implemented)
#include "pb_common.h"

namespace pb {
pb_status launch_srhd_c2p(pb_batch *, const void *, int, bool, double, hipStream_t)
{
    set_error("SRHD: not implemented in this build");
    return PB_EUNSUPPORTED;
}
}  // namespace pb

extern "C" {
pb_status con2prim(const void *, void *, int64_t, double, double, int32_t, int32_t, const pb_mlp *,
                   const void *, void *, void *, void *, void *)
{
    pb::set_error("con2prim: not implemented in this build");
    return PB_EUNSUPPORTED;
}
pb_status pb_mlp_create(pb_mlp **) { return PB_EUNSUPPORTED; }
pb_status pb_mlp_destroy(pb_mlp *) { return PB_OK; }
pb_status pb_mlp_set_params(pb_mlp *, const float *, const float *) { return PB_EUNSUPPORTED; }
pb_status pb_mlp_get_params(pb_mlp *, float *, float *) { return PB_EUNSUPPORTED; }
pb_status pb_mlp_forward(const pb_mlp *, const void *, void *, int64_t, void *) { return PB_EUNSUPPORTED; }
pb_status pb_mlp_grad(const pb_mlp *, const void *, const void *, int64_t, void *, void *, void *) { return PB_EUNSUPPORTED; }
pb_status pb_mlp_train_step(pb_mlp *, const void *, const void *, int64_t, float, float, float, float, int32_t, void *, void *) { return PB_EUNSUPPORTED; }
}
