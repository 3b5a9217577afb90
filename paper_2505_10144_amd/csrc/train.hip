// Fine-tuning (Sec. 4.1: the Gaussians are fine-tuned by backpropagation,
// starting from a converged model, Sec. 5): the image loss with its
// gradient, and an Adam step over a parameter array.
//
// Loss (the L1 + L2 reading of the objective): L = mean |I - I*| +
// 0.2 mean (I - I*)^2 over the RGB channels of every pixel of every view;
// dL/dI = (sign(I - I*) + 0.4 (I - I*)) / n on RGB, 0 on alpha.  The loss
// value is reduced deterministically: per-block partial sums in FP64, then
// one block adds them in a fixed order.
#include <string.h>

#include <cmath>

#include "vrs_internal.h"

namespace vrs {

constexpr int kLossThreads = 256;
constexpr int kLossBlocksPerView = 1024;

struct LossView {
    const float* img;     // [4][H][W]
    const float* target;  // [4][H][W]
    float* grad;          // [4][H][W]
    size_t plane;
};

struct LossViews {
    int n;
    double inv_n;  // 1 / (3 * total pixels)
    LossView v[VRS_MAX_VIEWS];
};

// Block (view v = blockIdx.y, part blockIdx.x): grid-stride over the view's
// pixels; writes its partial loss to partial[v * gridDim.x + blockIdx.x].
__global__ void __launch_bounds__(kLossThreads) k_loss_grad(LossViews views, double* __restrict__ partial) {
    const LossView& V = views.v[blockIdx.y];
    const float inv_n = float(views.inv_n);
    double acc = 0.0;
    for (size_t i = size_t(blockIdx.x) * kLossThreads + threadIdx.x; i < V.plane;
         i += size_t(gridDim.x) * kLossThreads) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float d = V.img[c * V.plane + i] - V.target[c * V.plane + i];
            const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
            V.grad[c * V.plane + i] = (sg + 0.4f * d) * inv_n;
            acc += double(fabsf(d)) + 0.2 * double(d) * double(d);
        }
        V.grad[3 * V.plane + i] = 0.f;
    }
    __shared__ double sh[kLossThreads / 64];
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < kLossThreads / 64; ++k) s += sh[k];
        partial[size_t(blockIdx.y) * gridDim.x + blockIdx.x] = s;
    }
}

// One block: the partials in a fixed order (per thread a strided slice, then
// the threads in order), times 1/n.
__global__ void __launch_bounds__(kLossThreads) k_loss_total(const double* __restrict__ partial, int count,
                                                             double inv_n, double* __restrict__ loss) {
    __shared__ double sh[kLossThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < count; i += kLossThreads) s += partial[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kLossThreads; ++k) t += sh[k];
        *loss = t * inv_n;
    }
}

// Adam with bias correction, one thread per element.
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, size_t count, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) {
        const float gi = g[i];
        const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
        const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

}  // namespace vrs

using namespace vrs;

extern "C" {

size_t vrs_loss_workspace_size(int32_t n_views) {
    return n_views < 1 ? 0 : size_t(n_views) * kLossBlocksPerView * sizeof(double);
}

int vrs_loss_l1l2(const vrs_camera* cams, int32_t n_views, const float* const* rgba, const float* const* target,
                  float* const* grad_rgba, double* loss_dev, void* ws, size_t ws_bytes, vrs_stream_t stream) {
    if (!cams || !rgba || !target || !grad_rgba || !loss_dev || n_views < 1 || n_views > VRS_MAX_VIEWS)
        return VRS_ERR_INVALID_ARG;
    if (!ws || ws_bytes < vrs_loss_workspace_size(n_views) || (reinterpret_cast<uintptr_t>(ws) & 7u))
        return VRS_ERR_INVALID_ARG;
    LossViews L;
    memset(&L, 0, sizeof(L));
    L.n = n_views;
    double total = 0.0;
    for (int v = 0; v < n_views; ++v) {
        if (cams[v].width < 1 || cams[v].height < 1 || !rgba[v] || !target[v] || !grad_rgba[v])
            return VRS_ERR_INVALID_ARG;
        L.v[v].img = rgba[v];
        L.v[v].target = target[v];
        L.v[v].grad = grad_rgba[v];
        L.v[v].plane = size_t(cams[v].width) * size_t(cams[v].height);
        total += 3.0 * double(L.v[v].plane);
    }
    L.inv_n = 1.0 / total;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double* partial = static_cast<double*>(ws);
    hipLaunchKernelGGL(k_loss_grad, dim3(kLossBlocksPerView, n_views), dim3(kLossThreads), 0, s, L, partial);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(kLossThreads), 0, s, partial, n_views * kLossBlocksPerView,
                       L.inv_n, loss_dev);
    return launch_status(hipGetLastError());
}

int vrs_adam_step(float* param, const float* grad, float* m, float* v, size_t count, float lr, float beta1,
                  float beta2, float eps, int32_t step, vrs_stream_t stream) {
    if (count == 0) return VRS_OK;
    if (!param || !grad || !m || !v || step < 1 || !(beta1 >= 0.f && beta1 < 1.f) ||
        !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f) || !std::isfinite(lr))
        return VRS_ERR_INVALID_ARG;
    const float c1 = float(1.0 - pow(double(beta1), double(step)));
    const float c2 = float(1.0 - pow(double(beta2), double(step)));
    const size_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(k_adam, dim3(unsigned(blocks < 65536 ? blocks : 65536)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), param, grad, m, v, count, lr, beta1, beta2, eps, c1,
                       c2);
    return launch_status(hipGetLastError());
}

}  // extern "C"
