// Variant-selector network on the GPU: dense layers with ReLU, masked mean
// squared error, and Adam, in FP32.
//
// The network predicts, from a request's features, the log-throughput of each
// scan variant; it is trained on the exhaustive autotuner's timings. It is a
// few thousand rows by 64 columns: every kernel here sums in a fixed order
// (no atomics), which keeps the GPU gradients reproducible and directly
// comparable with the FP64 reference.
#include <hip/hip_runtime.h>

#include "mpm_internal.h"

namespace mpm {

// Y[b, n] = act(bias[n] + sum_k X[b, k] W[k, n]); one thread per output, the
// layer's weights and bias staged in LDS once per workgroup (W[k, n] with n
// along the lanes: consecutive words), X[b, k] read as a broadcast.
template <bool Relu>
__global__ __launch_bounds__(1024) void dense_fwd(const float *__restrict__ X,
                                                  const float *__restrict__ W,
                                                  const float *__restrict__ bias,
                                                  float *__restrict__ Y, uint32_t B, uint32_t K,
                                                  uint32_t N)
{
    __shared__ float ws[MPM_MLP_HIDDEN * MPM_MLP_HIDDEN + MPM_MLP_HIDDEN];  // W then bias
    for (uint32_t i = threadIdx.x; i < K * N + N; i += blockDim.x)
        ws[i] = i < K * N ? W[i] : bias[i - K * N];
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)B * N)
        return;
    const uint32_t b = (uint32_t)(i / N), n = (uint32_t)(i % N);
    float acc = ws[K * N + n];
    const float *x = X + (uint64_t)b * K;
#pragma unroll 8
    for (uint32_t k = 0; k < K; ++k)
        acc = fmaf(x[k], ws[k * N + n], acc);
    Y[i] = Relu ? fmaxf(acc, 0.f) : acc;
}

// dX[b, k] = (sum_n dY[b, n] W[k, n]) * [A[b, k] > 0]: gradient through a
// layer into the previous ReLU output A. The weights are staged in LDS
// transposed (W[k, n] at n * K + k, k along the lanes), dY[b, n] is read as a
// broadcast.
__global__ __launch_bounds__(1024) void dense_bwd_data(const float *__restrict__ dY,
                                                       const float *__restrict__ W,
                                                       const float *__restrict__ A,
                                                       float *__restrict__ dX, uint32_t B,
                                                       uint32_t K, uint32_t N)
{
    __shared__ float wt[MPM_MLP_HIDDEN * MPM_MLP_HIDDEN];
    for (uint32_t i = threadIdx.x; i < K * N; i += blockDim.x) {
        const uint32_t k = i / N, n = i % N;
        wt[n * K + k] = W[i];
    }
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)B * K)
        return;
    const uint32_t b = (uint32_t)(i / K), k = (uint32_t)(i % K);
    float acc = 0.f;
    const float *dy = dY + (uint64_t)b * N;
#pragma unroll 8
    for (uint32_t n = 0; n < N; ++n)
        acc = fmaf(dy[n], wt[n * K + k], acc);
    dX[i] = A[i] > 0.f ? acc : 0.f;
}

// dW[k, n] = sum_b X[b, k] dY[b, n] and (row k == K) dbias[n] = sum_b dY[b, n],
// as a contraction over the batch in two deterministic stages. Stage one:
// workgroup (r, q) takes batch rows [r * WROWS, (r + 1) * WROWS) and gradient
// rows k = 17 q .. 17 q + 16. It stages in LDS, with coalesced loads, those
// 17 input columns of its batch rows (column K = 1 for the bias, columns past
// it 0; rows padded to XSTRIDE floats so each is four 16-byte words and one
// more) and their output gradients dY. Wave w sums batch rows
// [64 w, 64 w + 64) of the block, lane n column n, 17 accumulators per
// thread, with no branch in the loop; the four waves' sums are then added in
// wave order. With one row block the result goes straight to dW (dbias
// follows dW in the parameter vector); otherwise each block writes its
// partial gradient and stage two sums the partials in block order.
static const uint32_t WROWS = 256;
static const uint32_t WSLOTS = 17;   // gradient rows per workgroup quarter
static const uint32_t XSTRIDE = 20;  // staged floats per batch row (16-byte aligned)

// Copy count floats into LDS, 256 threads, sixteen loads in flight per thread
// before their stores (a load-store pair per step would wait out one memory
// round trip per element).
__device__ __forceinline__ void stage_lds(float *dst, const float *__restrict__ src, uint32_t count)
{
    constexpr uint32_t U = 16;
    uint32_t i = threadIdx.x;
    for (; i + (U - 1) * 256 < count; i += U * 256) {
        float v[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u)
            v[u] = src[i + u * 256];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u)
            dst[i + u * 256] = v[u];
    }
    for (; i < count; i += 256)
        dst[i] = src[i];
}

__global__ __launch_bounds__(256) void dense_bwd_weight(const float *__restrict__ X,
                                                        const float *__restrict__ dY,
                                                        float *__restrict__ out, uint32_t B,
                                                        uint32_t K, uint32_t N)
{
    __shared__ __align__(16) float xs[WROWS * XSTRIDE];
    __shared__ float ds[WROWS * MPM_MLP_HIDDEN];
    __shared__ float red[3][WSLOTS][MPM_MLP_HIDDEN];
    const uint32_t r0 = blockIdx.x * WROWS, k0 = blockIdx.y * WSLOTS;
    const uint32_t rows = min(WROWS, B - r0);
    {
        constexpr uint32_t U = 16;
        const uint32_t count = rows * XSTRIDE;
        for (uint32_t i0 = threadIdx.x; i0 < count; i0 += U * 256) {
            float v[U];
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t i = i0 + u * 256;
                const uint32_t b = i / XSTRIDE, k = k0 + i % XSTRIDE;
                v[u] = (i < count && k < K && i % XSTRIDE < WSLOTS)
                           ? X[(uint64_t)(r0 + b) * K + k]
                           : (k == K ? 1.f : 0.f);
            }
#pragma unroll
            for (uint32_t u = 0; u < U; ++u)
                if (i0 + u * 256 < count)
                    xs[i0 + u * 256] = v[u];
        }
    }
    stage_lds(ds, dY + (uint64_t)r0 * N, rows * N);
    __syncthreads();
    const uint32_t n = threadIdx.x & 63, w = threadIdx.x >> 6;
    float acc[WSLOTS];
#pragma unroll
    for (uint32_t j = 0; j < WSLOTS; ++j)
        acc[j] = 0.f;
    if (n < N) {
        const uint32_t b1 = min(rows, 64 * (w + 1));
#pragma unroll 4
        for (uint32_t b = 64 * w; b < b1; ++b) {
            const float d = ds[b * N + n];
            const float *x = xs + b * XSTRIDE;
#pragma unroll
            for (uint32_t j = 0; j < WSLOTS; ++j)
                acc[j] = fmaf(x[j], d, acc[j]);
        }
    }
    if (w > 0) {
#pragma unroll
        for (uint32_t j = 0; j < WSLOTS; ++j)
            red[w - 1][j][n] = acc[j];
    }
    __syncthreads();
    if (w == 0 && n < N) {
        float *o = out + (uint64_t)blockIdx.x * (K + 1) * N;
#pragma unroll
        for (uint32_t j = 0; j < WSLOTS; ++j) {
            const uint32_t k = k0 + j;
            if (k <= K)
                o[(uint64_t)k * N + n] = ((acc[j] + red[0][j][n]) + red[1][j][n]) + red[2][j][n];
        }
    }
}

// Stage two: dW[i] = sum over row blocks r (in order) of part[r][i].
__global__ void dense_bwd_weight_sum(const float *__restrict__ part, float *__restrict__ dW,
                                     uint32_t blocks, uint32_t count)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count)
        return;
    float s = 0.f;
    for (uint32_t r = 0; r < blocks; ++r)
        s += part[(uint64_t)r * count + i];
    dW[i] = s;
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
#pragma unroll 8
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
#pragma unroll 8
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
        const uint32_t nb = blocks_for((uint64_t)batch * N, 1024);
        if (l < 3)
            hipLaunchKernelGGL(dense_fwd<true>, dim3(nb), dim3(1024), 0, s, in, W, b, out, batch, K, N);
        else
            hipLaunchKernelGGL(dense_fwd<false>, dim3(nb), dim3(1024), 0, s, in, W, b, out, batch, K, N);
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
        // the gradient buffer this layer's data gradient will use is free
        // until then: it holds the partial weight gradients (at most
        // ceil(batch / 256) x 65 x 64 floats, within batch x 64 when there
        // is more than one row block)
        const uint32_t nrb = blocks_for(batch, WROWS);
        const uint32_t cnt = (K + 1) * N;
        float *part = nrb > 1 ? buf[l & 1] : dW;
        const uint32_t quarters = (K + 1 + WSLOTS - 1) / WSLOTS;
        hipLaunchKernelGGL(dense_bwd_weight, dim3(nrb, quarters), dim3(256), 0, s, A_prev, g, part,
                           batch, K, N);
        if (nrb > 1)
            hipLaunchKernelGGL(dense_bwd_weight_sum, dim3(blocks_for(cnt, 256)), dim3(256), 0, s,
                               part, dW, nrb, cnt);
        if (l > 0) {
            float *dX = buf[l & 1];
            hipLaunchKernelGGL(dense_bwd_data, dim3(blocks_for((uint64_t)batch * K, 1024)), dim3(1024),
                               0, s, g, W, A_prev, dX, batch, K, N);
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
