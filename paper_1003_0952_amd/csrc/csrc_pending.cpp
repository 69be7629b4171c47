// Entry points whose implementation is not yet in this build report
// CSRC_ERR_UNSUPPORTED.
#include "internal.h"

extern "C" {

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
