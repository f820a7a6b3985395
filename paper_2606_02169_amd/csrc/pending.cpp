// Entry points whose implementation is not in this build yet: they validate nothing and report
// MRMF_E_UNSUPPORTED.
#include "mrmf_internal.h"

extern "C" {
mrmf_status mrmf_adjoint_scratch_bytes(mrmf_plan, size_t*) { return MRMF_E_UNSUPPORTED; }
mrmf_status mrmf_adjoint_z(mrmf_plan, const void*, const double*, const void*, const void*, void*, double*,
                           void*, size_t, mrmf_stream) { return MRMF_E_UNSUPPORTED; }





mrmf_status mrmf_batch_create(int32_t, const mrmf_plan*, int32_t, mrmf_batch*) { return MRMF_E_UNSUPPORTED; }
void mrmf_batch_destroy(mrmf_batch) {}
mrmf_status mrmf_batch_total_elems(mrmf_batch, int64_t*) { return MRMF_E_UNSUPPORTED; }
mrmf_status mrmf_batch_offsets(mrmf_batch, int64_t*) { return MRMF_E_UNSUPPORTED; }
mrmf_status mrmf_batch_theta_offsets(mrmf_batch, int32_t*) { return MRMF_E_UNSUPPORTED; }
mrmf_status mrmf_batch_workspace_bytes(mrmf_batch, size_t*) { return MRMF_E_UNSUPPORTED; }
mrmf_status mrmf_batch_upload(mrmf_batch, void*, size_t, mrmf_stream) { return MRMF_E_UNSUPPORTED; }
mrmf_status mrmf_batch_matvec_c(mrmf_batch, const void*, const float*, const void*, void*, mrmf_stream) {
    return MRMF_E_UNSUPPORTED;
}
mrmf_status mrmf_batch_graph_capture(mrmf_batch, const void*, const float*, const void*, void*, mrmf_stream) {
    return MRMF_E_UNSUPPORTED;
}
mrmf_status mrmf_batch_graph_launch(mrmf_batch, mrmf_stream) { return MRMF_E_UNSUPPORTED; }
mrmf_status mrmf_batch_autotune(mrmf_batch, const void*, const float*, const void*, void*, mrmf_stream,
                                int32_t*) { return MRMF_E_UNSUPPORTED; }
mrmf_status mrmf_batch_set_shape(mrmf_batch, int32_t, int32_t) { return MRMF_E_UNSUPPORTED; }
}
