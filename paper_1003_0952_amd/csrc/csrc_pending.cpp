// Entry points whose implementation is not yet in this build report
// CSRC_ERR_UNSUPPORTED.
#include "internal.h"

extern "C" {

int csrc_batch_plan_create(int32_t, const int32_t *, const int32_t *const *, const int32_t *const *,
                           const int32_t *, int32_t, const csrc_batch_opts *, csrc_batch_plan **)
{ return CSRC_ERR_UNSUPPORTED; }
int csrc_batch_plan_destroy(csrc_batch_plan *) { return CSRC_OK; }
int64_t csrc_batch_workspace_bytes(const csrc_batch_plan *) { return -1; }
int csrc_batch_bind(const csrc_batch_plan *, const csrc_matrix *, const void *const *, const int64_t *,
                    void *const *, const int64_t *, void *, int64_t, void *) { return CSRC_ERR_UNSUPPORTED; }
int csrc_batch_run(const csrc_batch_plan *, int32_t, void *, int64_t, void *) { return CSRC_ERR_UNSUPPORTED; }
int csrc_spmv_batched(const csrc_batch_plan *, const csrc_matrix *, const void *const *, const int64_t *,
                      void *const *, const int64_t *, void *, int64_t, void *) { return CSRC_ERR_UNSUPPORTED; }
int csrc_spmv_t_batched(const csrc_batch_plan *, const csrc_matrix *, const void *const *, const int64_t *,
                        void *const *, const int64_t *, void *, int64_t, void *) { return CSRC_ERR_UNSUPPORTED; }
int csrc_batch_graph_create(const csrc_batch_plan *, int32_t, void *, int64_t, csrc_graph **)
{ return CSRC_ERR_UNSUPPORTED; }
int csrc_graph_launch(csrc_graph *, void *) { return CSRC_ERR_UNSUPPORTED; }
int csrc_graph_destroy(csrc_graph *) { return CSRC_OK; }
int64_t csrc_mlp_param_count(int32_t hidden, int32_t classes)
{
    return (int64_t)hidden * CSRC_NFEATURES + hidden + (int64_t)hidden * hidden + hidden +
           (int64_t)classes * hidden + classes;
}
int csrc_mlp_forward(int32_t, int32_t, int32_t, const float *, const float *, float *, float *, float *,
                     void *) { return CSRC_ERR_UNSUPPORTED; }
int csrc_mlp_backward(int32_t, int32_t, int32_t, const float *, const float *, const float *,
                      const float *, const int32_t *, float *, float *, void *) { return CSRC_ERR_UNSUPPORTED; }
int csrc_mlp_adam(int64_t, float *, const float *, float *, float *, int32_t, float, float, float, float,
                  void *) { return CSRC_ERR_UNSUPPORTED; }
}
