// L1 photometric loss and its gradient, reduced in a fixed order so that the
// loss value is identical on every run.  The mean is taken over `total`
// elements (the whole batch), of which one call sees n.
#include "ws_internal.h"

namespace ws {
namespace {

constexpr int kLossThreads = 256;
constexpr int kLossBlocks = 1024;

__global__ __launch_bounds__(kLossThreads) void k_l1_partial(const float* __restrict__ img,
                                                             const float* __restrict__ tgt, int64_t n, float inv_total,
                                                             float* __restrict__ dL, double* __restrict__ partial) {
    __shared__ double s_part[kLossThreads / kWave];
    double acc = 0.0;
    const int64_t stride = int64_t(gridDim.x) * kLossThreads;
    for (int64_t i = int64_t(blockIdx.x) * kLossThreads + threadIdx.x; i < n; i += stride) {
        const float d = img[i] - tgt[i];
        dL[i] = d > 0.f ? inv_total : (d < 0.f ? -inv_total : 0.f);
        acc += double(fabsf(d));
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) s_part[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kLossThreads / kWave; ++w) s += s_part[w];
        partial[blockIdx.x] = s;
    }
}

// One workgroup sums nb partial sums in a fixed order: thread t adds
// partial[t + k * kFinalThreads] for k = 0, 1, ... into kFinalUnroll
// accumulators by k mod kFinalUnroll (all of a round's loads in flight
// together), then the accumulators, the waves and the workgroup in order.
constexpr int kFinalThreads = 1024;
constexpr int kFinalUnroll = 8;

__global__ __launch_bounds__(kFinalThreads) void k_l1_final(const double* __restrict__ partial, int64_t nb,
                                                            int64_t total, const int32_t* d_status,
                                                            float* __restrict__ loss) {
    __shared__ double s_part[kFinalThreads / kWave];
    if (d_status && *d_status != 0) return;
    double acc[kFinalUnroll];
#pragma unroll
    for (int u = 0; u < kFinalUnroll; ++u) acc[u] = 0.0;
    constexpr int64_t kRound = int64_t(kFinalThreads) * kFinalUnroll;
    for (int64_t b = 0; b < nb; b += kRound) {
        double v[kFinalUnroll];
#pragma unroll
        for (int u = 0; u < kFinalUnroll; ++u) {
            const int64_t i = b + int64_t(u) * kFinalThreads + threadIdx.x;
            v[u] = i < nb ? partial[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kFinalUnroll; ++u) acc[u] += v[u];
    }
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < kFinalUnroll; ++u) a += acc[u];
    a = wave_sum(a);
    if (lane_id() == 0) s_part[threadIdx.x / kWave] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kFinalThreads / kWave; ++w) s += s_part[w];
        *loss = float(s / double(total));
    }
}

}  // namespace

size_t l1_loss_workspace(int64_t n) {
    (void)n;
    return align_up(kLossBlocks * sizeof(double));
}

hipError_t launch_l1_loss(const float* images, const float* targets, int64_t n, int64_t total, float* dL,
                          float* d_loss, void* ws, hipStream_t stream) {
    double* partial = static_cast<double*>(ws);
    // 1 / total rounded once from fp64, the value every gradient element takes
    const float inv_total = float(1.0 / double(total));
    hipLaunchKernelGGL(k_l1_partial, dim3(kLossBlocks), dim3(kLossThreads), 0, stream, images, targets, n, inv_total,
                       dL, partial);
    hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(kFinalThreads), 0, stream, partial, int64_t(kLossBlocks), total,
                       static_cast<const int32_t*>(nullptr), d_loss);
    return hipGetLastError();
}

void launch_l1_final(const double* partial, int64_t nb, int64_t total, const int32_t* d_status, float* loss,
                     hipStream_t stream) {
    hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(kFinalThreads), 0, stream, partial, nb, total, d_status, loss);
}

}  // namespace ws
