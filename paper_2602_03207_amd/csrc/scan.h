// Wait-free device-wide exclusive prefix sum (reduce, scan of the block sums,
// down-sweep): the hierarchical scheme of the paper's sort stage (Sec. 3.3.2),
// each level one dispatch, no workgroup ever waits for another.
//
//   k_scan_reduce<T, Loader>     block b sums items [b*kScanBlock, (b+1)*kScanBlock)
//   k_scan_partials<T>           one workgroup scans the block sums in place
//                                (exclusive) and optionally stores the total
//   k_scan_down<T, Loader, Writer>  block b re-reads its items, scans them and
//                                calls writer(i, exclusive_prefix, value)
//
// Loader:  __device__ T operator()(int64_t i) const   (i < n)
// Writer:  __device__ void operator()(int64_t i, T prefix, T value) const
// The number of items n may live in device memory (count pointer), so the
// launches can be sized for a capacity and captured in a graph.
#pragma once

#include "ws_internal.h"

namespace ws {

constexpr int kScanThreads = 256;
constexpr int kScanItemsPerThread = 16;
constexpr int kScanBlock = kScanThreads * kScanItemsPerThread;  // 4096 items per block
constexpr int kPartialThreads = 1024;

__device__ __forceinline__ int64_t scan_count(int64_t cap, const int64_t* d_n) {
    if (!d_n) return cap;
    const int64_t v = *d_n;
    return v < 0 ? 0 : (v < cap ? v : cap);
}

template <class T, class Loader>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(Loader ld, int64_t cap, const int64_t* d_n,
                                                              const int32_t* d_status, T* partials) {
    __shared__ T s_w[kScanThreads / kWave];
    if (d_status && *d_status != 0) return;
    const int64_t n = scan_count(cap, d_n);
    const int64_t base = int64_t(blockIdx.x) * kScanBlock;
    T sum = 0;
    // strided over the block so that a wave reads consecutive items
#pragma unroll
    for (int j = 0; j < kScanItemsPerThread; ++j) {
        const int64_t i = base + int64_t(j) * kScanThreads + threadIdx.x;
        if (i < n) sum += ld(i);
    }
    sum = wave_sum(sum);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
#pragma unroll
        for (int w = 0; w < kScanThreads / kWave; ++w) t += s_w[w];
        partials[blockIdx.x] = t;
    }
}

// One workgroup: exclusive scan of partials[0, nb) in place; total to *total_out.
template <class T>
__global__ __launch_bounds__(kPartialThreads) void k_scan_partials(T* partials, int64_t nb_cap, const int64_t* d_n,
                                                                   const int32_t* d_status, T* total_out) {
    __shared__ T s_scan[kPartialThreads / kWave + 1];
    __shared__ T s_carry;
    if (d_status && *d_status != 0) return;
    // number of blocks actually holding items
    const int64_t n = d_n ? scan_count(nb_cap * kScanBlock, d_n) : nb_cap * kScanBlock;
    const int64_t nb = d_n ? (n + kScanBlock - 1) / kScanBlock : nb_cap;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += kPartialThreads) {
        const int64_t b = b0 + threadIdx.x;
        const T v = b < nb ? partials[b] : T(0);
        T tot;
        const T ex = block_exclusive_scan<kPartialThreads>(v, s_scan, &tot);
        const T carry = s_carry;
        if (b < nb) partials[b] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total_out) *total_out = s_carry;
}

// Wave-striped: wave w owns items base + w*1024 + j*64 + lane (j < 16), so
// every load and store of the wave covers 64 consecutive items.
template <class T, class Loader, class Writer>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(Loader ld, Writer wr, int64_t cap, const int64_t* d_n,
                                                            const int32_t* d_status, const T* partials) {
    constexpr int kPerWave = kScanItemsPerThread * kWave;
    __shared__ T s_wave[kScanThreads / kWave];
    if (d_status && *d_status != 0) return;
    const int64_t n = scan_count(cap, d_n);
    const int64_t base = int64_t(blockIdx.x) * kScanBlock;
    if (base >= n) return;
    const int wave = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const int64_t wbase = base + int64_t(wave) * kPerWave + lane;
    T v[kScanItemsPerThread];
#pragma unroll
    for (int j = 0; j < kScanItemsPerThread; ++j) {
        const int64_t i = wbase + j * kWave;
        v[j] = i < n ? ld(i) : T(0);
    }
    // exclusive prefix of each item inside the wave's run of 1024
    T ex[kScanItemsPerThread];
    T carry = 0;
#pragma unroll
    for (int j = 0; j < kScanItemsPerThread; ++j) {
        const T inc = wave_inclusive_scan(v[j]);
        ex[j] = carry + inc - v[j];
        carry += __shfl(inc, kWave - 1, kWave);
    }
    if (lane == 0) s_wave[wave] = carry;
    __syncthreads();
    T off = partials[blockIdx.x];
    for (int w = 0; w < wave; ++w) off += s_wave[w];
#pragma unroll
    for (int j = 0; j < kScanItemsPerThread; ++j) {
        const int64_t i = wbase + j * kWave;
        if (i < n) wr(i, off + ex[j], v[j]);
    }
}

inline int64_t scan_blocks(int64_t cap) { return std::max<int64_t>((cap + kScanBlock - 1) / kScanBlock, 1); }

// Launch the three levels.  partials must hold scan_blocks(cap) values of T.
template <class T, class Loader, class Writer>
void launch_scan(const Loader& ld, const Writer& wr, int64_t cap, const int64_t* d_n, const int32_t* d_status,
                 T* partials, T* total_out, hipStream_t stream) {
    const int64_t nb = scan_blocks(cap);
    hipLaunchKernelGGL((k_scan_reduce<T, Loader>), dim3(uint32_t(nb)), dim3(kScanThreads), 0, stream, ld, cap, d_n,
                       d_status, partials);
    hipLaunchKernelGGL((k_scan_partials<T>), dim3(1), dim3(kPartialThreads), 0, stream, partials, nb, d_n, d_status,
                       total_out);
    hipLaunchKernelGGL((k_scan_down<T, Loader, Writer>), dim3(uint32_t(nb)), dim3(kScanThreads), 0, stream, ld, wr,
                       cap, d_n, d_status, partials);
}

}  // namespace ws
