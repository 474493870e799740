// Candidate-count model: y = W2 relu(W1 f + b1) + b2 over f_l = log(1 + s_l).
//
// The paper steers resources with an offline-trained model of data
// characteristics (Sections 5.2-5.3); here the model predicts log(1 + |C(q)|)
// from the bucket sizes the probe step produces, and the prediction only
// chooses each query's hash-set size class (results never depend on it).
// Training is FP32 (forward, hand-written backward, Adam); inference is BF16
// (inputs, weights and hidden activations rounded to bfloat16, FP32 sums).
// Packed parameters: W1 [H][L], b1 [H], W2 [H], b2.
#include "qw_internal.h"
#include "qw_mlp.h"

namespace qw {

constexpr int H = QW_MLP_HIDDEN;
constexpr int kSamples = 64;  // samples per workgroup in the gradient kernel

__global__ void features_kernel(const uint32_t *__restrict__ bsize, int64_t total,
                                float *__restrict__ feats)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        feats[i] = log1pf((float)bsize[i]);
}

qw_status launch_mlp_features(const uint32_t *bsize, int64_t Q, int32_t L, float *feats,
                              hipStream_t s)
{
    const int64_t total = Q * L;
    if (total <= 0) return QW_OK;
    int g = (int)std::min<int64_t>(65536, ceil_div(total, kBlock));
    features_kernel<<<g, kBlock, 0, s>>>(bsize, total, feats);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// 64 queries per workgroup round: their features go to LDS as bf16 (zero
// past L), then each wave runs the MFMA inference for 16 of them.
__global__ __launch_bounds__(kBlock) void mlp_predict_bf16_kernel(const float *__restrict__ params,
                                                                  int32_t L,
                                                                  const float *__restrict__ feats,
                                                                  int64_t B, float *__restrict__ out)
{
    static_assert(H == 64, "four 16-unit MFMA tiles");
    __shared__ __align__(16) uint16_t fsh[64 * (16 * kMlpMaxKs + 4)];
    __shared__ float sw[kMlpH * 16 * kMlpMaxKs + 2 * kMlpH + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ksteps = (L + 15) / 16;
    const int kp = 16 * ksteps, ld = kp + 4;  // padded rows (8-byte aligned)
    MlpLane m;
    mlp_lane_load(params, L, sw, m);
    for (int64_t q0 = (int64_t)blockIdx.x * 64; q0 < B; q0 += (int64_t)gridDim.x * 64) {
        for (int i = tid; i < 64 * kp; i += kBlock) {
            const int r = i / kp, k = i - r * kp;
            const int64_t q = q0 + r;
            fsh[r * ld + k] = k < L && q < B ? bf16_bits(feats[q * L + k]) : (uint16_t)0;
        }
        __syncthreads();
        const mlp_f4 y = mlp_predict16(fsh + wave * 16 * ld, ld, ksteps, m);
        if ((lane & 15) == 0)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t q = q0 + wave * 16 + (lane >> 4) * 4 + j;
                if (q < B) out[q] = y[j];
            }
        __syncthreads();  // fsh is rewritten by the next round
    }
}

qw_status launch_mlp_predict_bf16(const float *params, int32_t L, const float *feats, int64_t B,
                                  float *out, hipStream_t s)
{
    if (B <= 0) return QW_OK;
    if (L > 16 * kMlpMaxKs) return QW_EINVAL;
    const int g = (int)std::min<int64_t>(1024, ceil_div(B, 64));
    mlp_predict_bf16_kernel<<<g, kBlock, 0, s>>>(params, L, feats, B, out);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// Per-workgroup partial gradients of the mean squared error over kSamples
// samples; every parameter's partial is a fixed-order sum (deterministic).
__global__ __launch_bounds__(kBlock) void mlp_grad_partial_kernel(
    const float *__restrict__ params, int32_t L, const float *__restrict__ feats,
    const float *__restrict__ targets, int32_t B, float *__restrict__ partial /* [nblk][P+1] */)
{
    extern __shared__ float sm[];
    const int P = H * L + 2 * H + 1;
    float *f = sm;                       // [kSamples][L]
    float *dz = f + kSamples * L;        // [kSamples][H]
    float *act = dz + kSamples * H;      // [kSamples][H]
    float *dy = act + kSamples * H;      // [kSamples]
    float *r2 = dy + kSamples;           // [kSamples]
    const int s0 = blockIdx.x * kSamples;
    const int ns = min(kSamples, B - s0);
    for (int i = threadIdx.x; i < kSamples * L; i += kBlock) {
        const int s = i / L;
        f[i] = s < ns ? feats[(int64_t)(s0 + s) * L + (i - s * L)] : 0.f;
    }
    __syncthreads();
    const float *W1 = params, *b1 = params + H * L, *W2 = params + H * L + H;
    const float b2 = params[P - 1];
    // forward + backward to the hidden layer: thread t handles sample t % 64,
    // hidden units (t / 64) * 16 .. +16
    {
        const int s = threadIdx.x & (kSamples - 1);
        const int h0 = (threadIdx.x / kSamples) * (H / (kBlock / kSamples));
        for (int h = h0; h < h0 + H / (kBlock / kSamples); ++h) {
            float z = b1[h];
            for (int l = 0; l < L; ++l) z = fmaf(W1[h * L + l], f[s * L + l], z);
            act[s * H + h] = z > 0.f ? z : 0.f;
            dz[s * H + h] = z > 0.f ? 1.f : 0.f;  // relu mask for now
        }
    }
    __syncthreads();
    if (threadIdx.x < kSamples) {
        const int s = threadIdx.x;
        float y = b2;
        for (int h = 0; h < H; ++h) y = fmaf(W2[h], act[s * H + h], y);
        const float r = s < ns ? y - targets[s0 + s] : 0.f;
        dy[s] = s < ns ? 2.f * r / (float)B : 0.f;
        r2[s] = r * r / (float)B;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSamples * H; i += kBlock) {
        const int s = i / H, h = i - s * H;
        dz[i] = dz[i] * dy[s] * W2[h];
    }
    __syncthreads();
    float *out = partial + (int64_t)blockIdx.x * (P + 1);
    for (int p = threadIdx.x; p < P + 1; p += kBlock) {
        float g = 0.f;
        if (p < H * L) {  // dW1[h][l] = sum_s dz[s][h] f[s][l]
            const int h = p / L, l = p - h * L;
            for (int s = 0; s < kSamples; ++s) g += dz[s * H + h] * f[s * L + l];
        } else if (p < H * L + H) {  // db1
            const int h = p - H * L;
            for (int s = 0; s < kSamples; ++s) g += dz[s * H + h];
        } else if (p < H * L + 2 * H) {  // dW2[h] = sum_s dy[s] act[s][h]
            const int h = p - H * L - H;
            for (int s = 0; s < kSamples; ++s) g += dy[s] * act[s * H + h];
        } else if (p == P - 1) {  // db2
            for (int s = 0; s < kSamples; ++s) g += dy[s];
        } else {  // loss
            for (int s = 0; s < kSamples; ++s) g += r2[s];
        }
        out[p] = g;
    }
}

__global__ void mlp_grad_reduce_kernel(const float *__restrict__ partial, int nblk, int P,
                                       float *__restrict__ grad, float *__restrict__ loss)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P + 1; p += gridDim.x * blockDim.x) {
        float g = 0.f;
        for (int b = 0; b < nblk; ++b) g += partial[(int64_t)b * (P + 1) + p];
        if (p < P) grad[p] = g; else *loss = g;
    }
}

static DevBuf g_partial;  // scratch for partial gradients (one device per process)

qw_status launch_mlp_loss_grad(const float *params, int32_t L, const float *feats,
                               const float *targets, int32_t B, float *grad, float *loss,
                               hipStream_t s)
{
    const int P = H * L + 2 * H + 1;
    const int nblk = (int)ceil_div(B, kSamples);
    QW_TRY(g_partial.ensure(sizeof(float) * (size_t)nblk * (P + 1)));
    const size_t lds = sizeof(float) * (kSamples * L + 2 * kSamples * H + 2 * kSamples);
    mlp_grad_partial_kernel<<<nblk, kBlock, lds, s>>>(params, L, feats, targets, B,
                                                      g_partial.as<float>());
    QW_HIP(hipGetLastError());
    mlp_grad_reduce_kernel<<<(unsigned)ceil_div(P + 1, kBlock), kBlock, 0, s>>>(
        g_partial.as<float>(), nblk, P, grad, loss);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                            float *__restrict__ m, float *__restrict__ v, int32_t P, float lr,
                            float b1, float b2, float eps, float c1, float c2)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float mh = mi / c1, vh = vi / c2;
        p[i] -= lr * mh / (sqrtf(vh) + eps);
    }
}

qw_status launch_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t P,
                          int32_t step, float lr, float b1, float b2, float eps, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    adam_kernel<<<(unsigned)ceil_div(P, kBlock), kBlock, 0, s>>>(params, grad, m, v, P, lr, b1,
                                                                 b2, eps, c1, c2);
    QW_HIP(hipGetLastError());
    return QW_OK;
}

}  // namespace qw
