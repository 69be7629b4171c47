// Selector network on the GPU: a 12-H-H-K perceptron (ReLU, softmax
// cross-entropy) with forward, backward and Adam kernels (the host-side
// forward pass for inference is in csrc_mlp_host.cpp).  All FP32.  Parameters: W1[H,12] b1[H]
// W2[H,H] b2[H] W3[K,H] b3[K], row-major W[out, in].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "internal.h"

namespace csrc {

constexpr int kNF = CSRC_NFEATURES;

// One workgroup per sample; blockDim >= max(H, K).
__global__ void k_mlp_forward(int H, int K, int B, const float *__restrict__ p, const float *__restrict__ X,
                              float *__restrict__ act, float *__restrict__ logits, float *__restrict__ probs)
{
    extern __shared__ float sm[];
    float *f = sm;            // 12
    float *h1 = f + kNF;      // H
    float *h2 = h1 + H;       // H
    float *z = h2 + H;        // K
    const MlpLayout L = mlp_layout(H, K);
    const int b = blockIdx.x, t = threadIdx.x;
    if (t < kNF) f[t] = X[(int64_t)b * kNF + t];
    __syncthreads();
    if (t < H) {
        float s = p[L.b1 + t];
        for (int i = 0; i < kNF; ++i) s += p[L.W1 + (int64_t)t * kNF + i] * f[i];
        h1[t] = s > 0.f ? s : 0.f;
    }
    __syncthreads();
    if (t < H) {
        float s = p[L.b2 + t];
        for (int i = 0; i < H; ++i) s += p[L.W2 + (int64_t)t * H + i] * h1[i];
        h2[t] = s > 0.f ? s : 0.f;
    }
    __syncthreads();
    if (t < K) {
        float s = p[L.b3 + t];
        for (int i = 0; i < H; ++i) s += p[L.W3 + (int64_t)t * H + i] * h2[i];
        z[t] = s;
    }
    __syncthreads();
    if (t < K) {
        float mx = z[0];
        for (int i = 1; i < K; ++i) mx = fmaxf(mx, z[i]);
        float den = 0.f;
        for (int i = 0; i < K; ++i) den += expf(z[i] - mx);
        logits[(int64_t)b * K + t] = z[t];
        probs[(int64_t)b * K + t] = expf(z[t] - mx) / den;
    }
    if (act && t < H) {
        act[(int64_t)b * 2 * H + t] = h1[t];
        act[(int64_t)b * 2 * H + H + t] = h2[t];
    }
}

// Per-sample deltas: d3 = (p - onehot)/B, d2 = (W3^T d3) * [h2 > 0],
// d1 = (W2^T d2) * [h1 > 0], stored as work[b] = (d3[K], d2[H], d1[H]).
__global__ void k_mlp_deltas(int H, int K, int B, const float *__restrict__ p, const float *__restrict__ act,
                             const float *__restrict__ probs, const int32_t *__restrict__ labels,
                             float *__restrict__ work)
{
    extern __shared__ float sm[];
    float *d3 = sm;        // K
    float *d2 = d3 + K;    // H
    const MlpLayout L = mlp_layout(H, K);
    const int b = blockIdx.x, t = threadIdx.x;
    const int64_t wb = (int64_t)b * (2 * H + K);
    if (t < K) {
        float v = probs[(int64_t)b * K + t] - (labels[b] == t ? 1.f : 0.f);
        v /= (float)B;
        d3[t] = v;
        work[wb + t] = v;
    }
    __syncthreads();
    if (t < H) {
        float s = 0.f;
        for (int k = 0; k < K; ++k) s += p[L.W3 + (int64_t)k * H + t] * d3[k];
        s = act[(int64_t)b * 2 * H + H + t] > 0.f ? s : 0.f;
        d2[t] = s;
        work[wb + K + t] = s;
    }
    __syncthreads();
    if (t < H) {
        float s = 0.f;
        for (int h = 0; h < H; ++h) s += p[L.W2 + (int64_t)h * H + t] * d2[h];
        s = act[(int64_t)b * 2 * H + t] > 0.f ? s : 0.f;
        work[wb + K + H + t] = s;
    }
}

// One thread per parameter: its gradient summed over the batch in order.
__global__ void k_mlp_grads(int H, int K, int B, const float *__restrict__ X, const float *__restrict__ act,
                            const float *__restrict__ work, float *__restrict__ g)
{
    const MlpLayout L = mlp_layout(H, K);
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= L.total) return;
    const int W = 2 * H + K;
    float s = 0.f;
    if (q >= L.b3) {                       // b3[k]
        const int k = (int)(q - L.b3);
        for (int b = 0; b < B; ++b) s += work[(int64_t)b * W + k];
    } else if (q >= L.W3) {                // W3[k][h] = sum d3[k] h2[h]
        const int k = (int)((q - L.W3) / H), h = (int)((q - L.W3) % H);
        for (int b = 0; b < B; ++b) s += work[(int64_t)b * W + k] * act[(int64_t)b * 2 * H + H + h];
    } else if (q >= L.b2) {                // b2[h]
        const int h = (int)(q - L.b2);
        for (int b = 0; b < B; ++b) s += work[(int64_t)b * W + K + h];
    } else if (q >= L.W2) {                // W2[h][i] = sum d2[h] h1[i]
        const int h = (int)((q - L.W2) / H), i = (int)((q - L.W2) % H);
        for (int b = 0; b < B; ++b) s += work[(int64_t)b * W + K + h] * act[(int64_t)b * 2 * H + i];
    } else if (q >= L.b1) {                // b1[h]
        const int h = (int)(q - L.b1);
        for (int b = 0; b < B; ++b) s += work[(int64_t)b * W + K + H + h];
    } else {                               // W1[h][f] = sum d1[h] x[f]
        const int h = (int)(q / kNF), f = (int)(q % kNF);
        for (int b = 0; b < B; ++b) s += work[(int64_t)b * W + K + H + h] * X[(int64_t)b * kNF + f];
    }
    g[q] = s;
}

// Mean cross-entropy: one workgroup, fixed reduction order.
__global__ void k_mlp_loss(int K, int B, const float *__restrict__ probs, const int32_t *__restrict__ labels,
                           float *__restrict__ loss)
{
    __shared__ float part[256];
    float s = 0.f;
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        const float pv = probs[(int64_t)b * K + labels[b]];
        s += -logf(fmaxf(pv, 1e-30f));
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = part[0] / (float)B;
}

__global__ void k_adam(int64_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

static int mlp_block(int H, int K)
{
    int t = H > K ? H : K;
    if (t < kNF) t = kNF;
    return ((t + 63) / 64) * 64;
}

}  // namespace csrc

extern "C" int csrc_mlp_forward(int32_t H, int32_t K, int32_t B, const float *params, const float *feats, float *act,
                                float *logits, float *probs, void *stream)
{
    using namespace csrc;
    if (!mlp_shape_ok(H, K, B) || (B > 0 && (!params || !feats || !logits || !probs))) return CSRC_ERR_ARG;
    if (B == 0) return CSRC_OK;
    const size_t sm = (size_t)(kNF + 2 * H + K) * sizeof(float);
    k_mlp_forward<<<B, mlp_block(H, K), sm, static_cast<hipStream_t>(stream)>>>(H, K, B, params, feats, act, logits,
                                                                                probs);
    return hip_status(hipGetLastError());
}

extern "C" int csrc_mlp_backward(int32_t H, int32_t K, int32_t B, const float *params, const float *feats,
                                 const float *act, const float *probs, const int32_t *labels, float *grads,
                                 float *loss, float *work, void *stream)
{
    using namespace csrc;
    if (!mlp_shape_ok(H, K, B) || !grads) return CSRC_ERR_ARG;
    if (B > 0 && (!params || !feats || !act || !probs || !labels || !work)) return CSRC_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t P = mlp_layout(H, K).total;
    if (B > 0) {
        k_mlp_deltas<<<B, mlp_block(H, K), (size_t)(K + H) * sizeof(float), s>>>(H, K, B, params, act, probs, labels,
                                                                                 work);
        if (loss) k_mlp_loss<<<1, 256, 0, s>>>(K, B, probs, labels, loss);
    }
    k_mlp_grads<<<(unsigned)((P + 255) / 256), 256, 0, s>>>(H, K, B, feats, act, work, grads);
    return hip_status(hipGetLastError());
}

extern "C" int csrc_mlp_adam(int64_t count, float *params, const float *grads, float *m, float *v, int32_t step,
                             float lr, float beta1, float beta2, float eps, void *stream)
{
    using namespace csrc;
    if (count < 0 || step < 1 || (count > 0 && (!params || !grads || !m || !v))) return CSRC_ERR_ARG;
    if (count == 0) return CSRC_OK;
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    const int grid = (int)std::min<int64_t>(1024, (count + 255) / 256);
    k_adam<<<grid, 256, 0, static_cast<hipStream_t>(stream)>>>(count, params, grads, m, v, lr, beta1, beta2, eps, c1,
                                                               c2);
    return hip_status(hipGetLastError());
}
