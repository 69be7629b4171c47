// Host side of the selector network: parameter count and the forward pass
// used for inference (csrc_mlp_predict_host), FP32, same parameter layout as
// the device kernels: W1[H,12] b1[H] W2[H,H] b2[H] W3[K,H] b3[K], row-major
// W[out, in].
#include <cstdint>
#include <vector>

#include "internal.h"

extern "C" int64_t csrc_mlp_param_count(int32_t hidden, int32_t classes)
{
    if (!csrc::mlp_shape_ok(hidden, classes, 0)) return -1;
    return csrc::mlp_layout(hidden, classes).total;
}

extern "C" int csrc_mlp_predict_host(int32_t H, int32_t K, const float *p, const float *mean, const float *scale,
                                     const float *features, int32_t *cls)
{
    using namespace csrc;
    if (!mlp_shape_ok(H, K, 1) || !p || !mean || !scale || !features || !cls) return CSRC_ERR_ARG;
    const MlpLayout L = mlp_layout(H, K);
    float f[kMlpFeatures];
    for (int i = 0; i < kMlpFeatures; ++i) f[i] = (features[i] - mean[i]) / (scale[i] != 0.f ? scale[i] : 1.f);
    std::vector<float> h1(H), h2(H);
    for (int h = 0; h < H; ++h) {
        float s = p[L.b1 + h];
        for (int i = 0; i < kMlpFeatures; ++i) s += p[L.W1 + (int64_t)h * kMlpFeatures + i] * f[i];
        h1[h] = s > 0.f ? s : 0.f;
    }
    for (int h = 0; h < H; ++h) {
        float s = p[L.b2 + h];
        for (int i = 0; i < H; ++i) s += p[L.W2 + (int64_t)h * H + i] * h1[i];
        h2[h] = s > 0.f ? s : 0.f;
    }
    int best = 0;
    float bz = 0.f;
    for (int k = 0; k < K; ++k) {
        float s = p[L.b3 + k];
        for (int i = 0; i < H; ++i) s += p[L.W3 + (int64_t)k * H + i] * h2[i];
        if (k == 0 || s > bz) { bz = s; best = k; }
    }
    *cls = best;
    return CSRC_OK;
}
