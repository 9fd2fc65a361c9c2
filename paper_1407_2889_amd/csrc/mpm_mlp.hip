// Variant-selector network on the GPU: dense layers with ReLU, masked mean
// squared error, and Adam, in FP32.
//
// The network predicts, from a request's features, the log-throughput of each
// scan variant; it is trained on the exhaustive autotuner's timings. It is a
// few thousand rows by 64 columns: every kernel here is a plain per-element
// or per-column loop with deterministic summation order (no atomics), which
// keeps the GPU gradients reproducible and directly comparable with the FP64
// reference.
#include <hip/hip_runtime.h>

#include "mpm_internal.h"

namespace mpm {

// Y[b, n] = act(bias[n] + sum_k X[b, k] W[k, n]); one thread per output.
template <bool Relu>
__global__ void dense_fwd(const float *__restrict__ X, const float *__restrict__ W,
                          const float *__restrict__ bias, float *__restrict__ Y, uint32_t B,
                          uint32_t K, uint32_t N)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)B * N)
        return;
    const uint32_t b = (uint32_t)(i / N), n = (uint32_t)(i % N);
    float acc = bias[n];
    const float *x = X + (uint64_t)b * K;
    for (uint32_t k = 0; k < K; ++k)
        acc = fmaf(x[k], W[(uint64_t)k * N + n], acc);
    Y[i] = Relu ? fmaxf(acc, 0.f) : acc;
}

// dX[b, k] = (sum_n dY[b, n] W[k, n]) * [A[b, k] > 0]: gradient through a
// layer into the previous ReLU output A.
__global__ void dense_bwd_data(const float *__restrict__ dY, const float *__restrict__ W,
                               const float *__restrict__ A, float *__restrict__ dX, uint32_t B,
                               uint32_t K, uint32_t N)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)B * K)
        return;
    const uint32_t b = (uint32_t)(i / K), k = (uint32_t)(i % K);
    float acc = 0.f;
    const float *dy = dY + (uint64_t)b * N;
    const float *w = W + (uint64_t)k * N;
    for (uint32_t n = 0; n < N; ++n)
        acc = fmaf(dy[n], w[n], acc);
    dX[i] = A[i] > 0.f ? acc : 0.f;
}

// dW[k, n] = sum_b X[b, k] dY[b, n] and (row k == K) dbias[n] = sum_b dY[b, n].
// Block (k, n-tile of 64): 4 waves split the batch, lane = column; partial
// sums combined in LDS in a fixed order.
__global__ __launch_bounds__(256) void dense_bwd_weight(const float *__restrict__ X,
                                                        const float *__restrict__ dY,
                                                        float *__restrict__ dW,
                                                        float *__restrict__ dbias, uint32_t B,
                                                        uint32_t K, uint32_t N)
{
    __shared__ float part[4][64];
    const uint32_t k = blockIdx.x;  // 0..K (K = bias row)
    const uint32_t n = blockIdx.y * 64 + (threadIdx.x & 63);
    const uint32_t w = threadIdx.x >> 6;
    float acc = 0.f;
    if (n < N) {
        for (uint32_t b = w; b < B; b += 4) {
            const float x = k < K ? X[(uint64_t)b * K + k] : 1.f;
            acc = fmaf(x, dY[(uint64_t)b * N + n], acc);
        }
    }
    part[w][threadIdx.x & 63] = acc;
    __syncthreads();
    if (w == 0 && n < N) {
        const float s = (part[0][threadIdx.x] + part[1][threadIdx.x]) +
                        (part[2][threadIdx.x] + part[3][threadIdx.x]);
        if (k < K)
            dW[(uint64_t)k * N + n] = s;
        else
            dbias[n] = s;
    }
}

// Masked MSE over B x N: loss = sum M (Y - T)^2 / sum M and
// dY = 2 M (Y - T) / sum M. One workgroup, fixed reduction order.
__global__ __launch_bounds__(1024) void mse_grad(const float *__restrict__ Y,
                                                 const float *__restrict__ T,
                                                 const float *__restrict__ M,
                                                 float *__restrict__ dY, float *__restrict__ loss,
                                                 uint64_t count)
{
    __shared__ float s_m[1024], s_e[1024];
    float sm = 0.f, se = 0.f;
    for (uint64_t i = threadIdx.x; i < count; i += 1024) {
        const float d = Y[i] - T[i];
        sm += M[i];
        se = fmaf(M[i] * d, d, se);
    }
    s_m[threadIdx.x] = sm;
    s_e[threadIdx.x] = se;
    __syncthreads();
    for (uint32_t o = 512; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s_m[threadIdx.x] += s_m[threadIdx.x + o];
            s_e[threadIdx.x] += s_e[threadIdx.x + o];
        }
        __syncthreads();
    }
    const float tot = s_m[0] > 0.f ? s_m[0] : 1.f;
    if (threadIdx.x == 0 && loss)
        *loss = s_e[0] / tot;
    const float scale = 2.f / tot;
    for (uint64_t i = threadIdx.x; i < count; i += 1024)
        dY[i] = scale * M[i] * (Y[i] - T[i]);
}

// Adam with bias correction (t counts from 1).
__global__ void adam_kernel(float *__restrict__ th, const float *__restrict__ g,
                            float *__restrict__ m, float *__restrict__ v, uint32_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static const uint32_t LAYERS[5] = {MPM_MLP_IN, MPM_MLP_HIDDEN, MPM_MLP_HIDDEN, MPM_MLP_HIDDEN,
                                   MPM_MLP_OUT};

static uint64_t layer_off(int l)  // offset of W_l in the parameter vector
{
    uint64_t o = 0;
    for (int i = 0; i < l; ++i)
        o += (uint64_t)LAYERS[i] * LAYERS[i + 1] + LAYERS[i + 1];
    return o;
}

static mpm_status hip_check(const char *where)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(MPM_EHIP, "%s: %s", where, hipGetErrorString(e));
    return MPM_OK;
}

static uint32_t blocks_for(uint64_t n, uint32_t t) { return (uint32_t)((n + t - 1) / t); }

}  // namespace mpm

using namespace mpm;

extern "C" {

uint64_t mpm_mlp_act_floats(uint32_t batch) { return 3ull * batch * MPM_MLP_HIDDEN; }

mpm_status mpm_mlp_forward(const float *d_theta, const float *d_x, uint32_t batch, float *d_act,
                           float *d_y, void *stream)
{
    if (!d_theta || !d_x || !d_act || !d_y || batch == 0)
        return fail(MPM_EINVAL, "mpm_mlp_forward: null argument or empty batch");
    hipStream_t s = (hipStream_t)stream;
    const float *in = d_x;
    for (int l = 0; l < 4; ++l) {
        const uint32_t K = LAYERS[l], N = LAYERS[l + 1];
        const float *W = d_theta + layer_off(l);
        const float *b = W + (uint64_t)K * N;
        float *out = l < 3 ? d_act + (uint64_t)l * batch * MPM_MLP_HIDDEN : d_y;
        const uint32_t nb = blocks_for((uint64_t)batch * N, 256);
        if (l < 3)
            hipLaunchKernelGGL(dense_fwd<true>, dim3(nb), dim3(256), 0, s, in, W, b, out, batch, K, N);
        else
            hipLaunchKernelGGL(dense_fwd<false>, dim3(nb), dim3(256), 0, s, in, W, b, out, batch, K, N);
        in = out;
    }
    return hip_check("mpm_mlp_forward");
}

mpm_status mpm_mlp_loss_grad(const float *d_y, const float *d_t, const float *d_mask, uint32_t batch,
                             float *d_dy, float *d_loss, void *stream)
{
    if (!d_y || !d_t || !d_mask || !d_dy || batch == 0)
        return fail(MPM_EINVAL, "mpm_mlp_loss_grad: null argument or empty batch");
    hipLaunchKernelGGL(mse_grad, dim3(1), dim3(1024), 0, (hipStream_t)stream, d_y, d_t, d_mask, d_dy,
                       d_loss, (uint64_t)batch * MPM_MLP_OUT);
    return hip_check("mpm_mlp_loss_grad");
}

mpm_status mpm_mlp_backward(const float *d_theta, const float *d_x, const float *d_act,
                            const float *d_dy, uint32_t batch, float *d_grad, float *d_tmp,
                            void *stream)
{
    if (!d_theta || !d_x || !d_act || !d_dy || !d_grad || !d_tmp || batch == 0)
        return fail(MPM_EINVAL, "mpm_mlp_backward: null argument or empty batch");
    hipStream_t s = (hipStream_t)stream;
    // d_tmp holds two batch x 64 gradient buffers used in turn.
    float *buf[2] = {d_tmp, d_tmp + (uint64_t)batch * MPM_MLP_HIDDEN};
    const float *g = d_dy;
    for (int l = 3; l >= 0; --l) {
        const uint32_t K = LAYERS[l], N = LAYERS[l + 1];
        const float *W = d_theta + layer_off(l);
        const float *A_prev = l == 0 ? d_x : d_act + (uint64_t)(l - 1) * batch * MPM_MLP_HIDDEN;
        float *dW = d_grad + layer_off(l);
        float *db = dW + (uint64_t)K * N;
        hipLaunchKernelGGL(dense_bwd_weight, dim3(K + 1, blocks_for(N, 64)), dim3(256), 0, s, A_prev,
                           g, dW, db, batch, K, N);
        if (l > 0) {
            float *dX = buf[l & 1];
            hipLaunchKernelGGL(dense_bwd_data, dim3(blocks_for((uint64_t)batch * K, 256)), dim3(256), 0,
                               s, g, W, A_prev, dX, batch, K, N);
            g = dX;
        }
    }
    return hip_check("mpm_mlp_backward");
}

mpm_status mpm_mlp_adam(float *d_theta, const float *d_grad, float *d_m, float *d_v, uint32_t n,
                        uint32_t t, float lr, float b1, float b2, float eps, void *stream)
{
    if (!d_theta || !d_grad || !d_m || !d_v || n == 0 || t == 0)
        return fail(MPM_EINVAL, "mpm_mlp_adam: null argument, n == 0 or t == 0");
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream,
                       d_theta, d_grad, d_m, d_v, n, lr, b1, b2, eps, c1, c2);
    return hip_check("mpm_mlp_adam");
}

}  // extern "C"
