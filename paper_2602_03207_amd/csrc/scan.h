// Device-wide exclusive prefix sums.
//
// Two schedules, chosen by the number of blocks:
//  * one pass (up to kOnePassMaxBlocks blocks, or any number for a sparse
//    scan, whose live count read from device memory is typically far below
//    the capacity the grid is sized for): every block scans its items in
//    registers, publishes its sum, reads its predecessors' published sums
//    (a decoupled look-back: one wave reads 64 predecessors per round trip
//    and stops at the first inclusive prefix) and writes its results.  Block
//    b scans chunk b and waits only for blocks with smaller indices; the
//    smallest unfinished block is always running, since each XCD starts its
//    workgroups in index order (its resources can only be held by blocks with
//    smaller indices, which have finished).  The wait is bounded
//    (WS_ERR_SPIN_LIMIT on expiry).  One read of the items, two launches
//    (clearing the published sums, the pass).
//  * wait-free (larger dense inputs): the hierarchical scan of the paper's sort
//    stage (Sec. 3.3.2) -- reduce, one-workgroup scan of the block sums,
//    down-sweep -- each level one dispatch, no workgroup ever waits for
//    another.
//
// Loader:  using Item = ...;                    what the writer needs of item i
//          __device__ Item operator()(int64_t i) const      (0 <= i < n)
//          __device__ static T value(const Item&)           the item's summand
// Writer:  __device__ void operator()(int64_t i, T prefix, const Item&) const
// Every thread loads all of its items before it uses any (indices past the
// end are clamped to the last item and their values replaced by zero), so a
// block waits for one round of memory latency, not one per item.
// The number of items n may live in device memory (count pointer), so the
// launches can be sized for a capacity and captured in a graph.
#pragma once

#include "ws_internal.h"

namespace ws {

// Blocks of 256 threads with ITEMS items each (a template parameter of every
// kernel and launcher: few large blocks shorten the look-back of an input
// whose items are all present; more, smaller blocks suit a sparse input whose
// items take dependent loads).
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;  // default: 4096 items per block
constexpr int kPartialThreads = 1024;

__device__ __forceinline__ int64_t scan_count(int64_t cap, const int64_t* d_n) {
    if (!d_n) return cap;
    const int64_t v = *d_n;
    return v < 0 ? 0 : (v < cap ? v : cap);
}

template <class T, int ITEMS, class Loader>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(Loader ld, int64_t cap, const int64_t* d_n,
                                                              const int32_t* d_status, T* partials) {
    __shared__ T s_w[kScanThreads / kWave];
    if (d_status && *d_status != 0) return;
    const int64_t n = scan_count(cap, d_n);
    const int64_t base = int64_t(blockIdx.x) * (kScanThreads * ITEMS);
    if (base >= n) {
        if (threadIdx.x == 0) partials[blockIdx.x] = T(0);
        return;
    }
    // strided over the block so that a wave reads consecutive items
    typename Loader::Item it[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = base + int64_t(j) * kScanThreads + threadIdx.x;
        it[j] = ld(i < n ? i : n - 1);
    }
    T sum = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = base + int64_t(j) * kScanThreads + threadIdx.x;
        sum += i < n ? Loader::value(it[j]) : T(0);
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
template <class T, int ITEMS>
__global__ __launch_bounds__(kPartialThreads) void k_scan_partials(T* partials, int64_t nb_cap, const int64_t* d_n,
                                                                   const int32_t* d_status, T* total_out) {
    __shared__ T s_scan[kPartialThreads / kWave + 1];
    __shared__ T s_carry;
    if (d_status && *d_status != 0) return;
    // number of blocks actually holding items
    const int64_t n = d_n ? scan_count(nb_cap * (kScanThreads * ITEMS), d_n) : nb_cap * (kScanThreads * ITEMS);
    const int64_t nb = d_n ? (n + (kScanThreads * ITEMS) - 1) / (kScanThreads * ITEMS) : nb_cap;
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

// Wave-striped: wave w owns items base + w*64*ITEMS + j*64 + lane (j < ITEMS),
// so every load and store of the wave covers 64 consecutive items.
template <class T, int ITEMS, class Loader, class Writer>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(Loader ld, Writer wr, int64_t cap, const int64_t* d_n,
                                                            const int32_t* d_status, const T* partials) {
    constexpr int kPerWave = ITEMS * kWave;
    __shared__ T s_wave[kScanThreads / kWave];
    if (d_status && *d_status != 0) return;
    const int64_t n = scan_count(cap, d_n);
    const int64_t base = int64_t(blockIdx.x) * (kScanThreads * ITEMS);
    if (base >= n) return;
    const int wave = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const int64_t wbase = base + int64_t(wave) * kPerWave + lane;
    typename Loader::Item it[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = wbase + j * kWave;
        it[j] = ld(i < n ? i : n - 1);
    }
    T v[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) v[j] = wbase + j * kWave < n ? Loader::value(it[j]) : T(0);
    // exclusive prefix of each item inside the wave's run of 1024
    T ex[ITEMS];
    T carry = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const T inc = wave_inclusive_scan(v[j]);
        ex[j] = carry + inc - v[j];
        carry += last_lane(inc);
    }
    if (lane == 0) s_wave[wave] = carry;
    __syncthreads();
    T off = partials[blockIdx.x];
    for (int w = 0; w < wave; ++w) off += s_wave[w];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = wbase + j * kWave;
        if (i < n) wr(i, off + ex[j], it[j]);
    }
}

inline int64_t scan_blocks(int64_t cap, int items) {
    const int64_t block = int64_t(kScanThreads) * items;
    return std::max<int64_t>((cap + block - 1) / block, 1);
}

// ---------------------------------------------------------- one pass

constexpr int64_t kOnePassMaxBlocks = 1024;
constexpr uint64_t kScanAgg = uint64_t(1) << 62;
constexpr uint64_t kScanInc = uint64_t(2) << 62;
constexpr uint64_t kScanVal = (uint64_t(1) << 62) - 1;

template <int Threads>
__global__ __launch_bounds__(Threads) void k_scan_clear(uint64_t* status, int64_t nb) {
    for (int64_t i = threadIdx.x; i < nb; i += Threads) status[i] = 0;
}

template <class T, int ITEMS, class Loader, class Writer>
__global__ __launch_bounds__(kScanThreads) void k_scan_onepass(Loader ld, Writer wr, int64_t cap, const int64_t* d_n,
                                                               const int32_t* d_status, uint64_t* status,
                                                               T* total_out) {
    constexpr int kPerWave = ITEMS * kWave;
    __shared__ T s_wave[kScanThreads / kWave];
    __shared__ T s_excl;
    if (d_status && *d_status != 0) return;
    const int64_t n = scan_count(cap, d_n);
    const int64_t nb = (n + (kScanThreads * ITEMS) - 1) / (kScanThreads * ITEMS);
    if (nb == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && total_out) *total_out = T(0);
        return;
    }
    // blocks past the live ones leave at once
    if (int64_t(blockIdx.x) >= nb) return;
    const int64_t b = blockIdx.x;
    const int wave = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const int64_t wbase = b * (kScanThreads * ITEMS) + int64_t(wave) * kPerWave + lane;
    typename Loader::Item it[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = wbase + j * kWave;
        it[j] = ld(i < n ? i : n - 1);
    }
    T v[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) v[j] = wbase + j * kWave < n ? Loader::value(it[j]) : T(0);
    T ex[ITEMS];
    T carry = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const T inc = wave_inclusive_scan(v[j]);
        ex[j] = carry + inc - v[j];
        carry += last_lane(inc);
    }
    if (lane == 0) s_wave[wave] = carry;
    __syncthreads();
    T block_sum = 0, woff = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        if (w < wave) woff += s_wave[w];
        block_sum += s_wave[w];
    }
    if (wave == 0) {
        if (lane == 0) store_agent(&status[b], (b == 0 ? kScanInc : kScanAgg) | uint64_t(block_sum));
        T excl = 0;
        if (b > 0) {
            int64_t k = b - 1;  // lane l reads predecessor k - l
            uint32_t spins = 0;
            while (true) {
                const int64_t kk = k - int64_t(lane);
                uint64_t st = kk >= 0 ? load_agent(&status[kk]) : kScanInc;
                uint64_t need = 0, incm = 0;
                while (true) {
                    incm = __ballot((st >> 62) == 2);
                    const uint64_t zero = __ballot((st >> 62) == 0);
                    // lanes up to and including the first inclusive prefix
                    need = incm ? ((incm & (~incm + 1)) << 1) - 1 : ~uint64_t(0);
                    if ((zero & need) == 0) break;
                    if (++spins > kSpinLimit) {
                        if (lane == 0) atomicExch(const_cast<int32_t*>(d_status), int32_t(WS_ERR_SPIN_LIMIT));
                        need = 0;
                        incm = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    if ((st >> 62) == 0) st = load_agent(&status[kk]);
                }
                const T part = ((need >> lane) & 1) ? T(st & kScanVal) : T(0);
                excl += wave_sum(part);
                if (incm) break;
                k -= kWave;
            }
            if (lane == 0) store_agent(&status[b], kScanInc | uint64_t(excl + block_sum));
        }
        if (lane == 0) {
            s_excl = excl;
            if (b == nb - 1 && total_out) *total_out = excl + block_sum;
        }
    }
    __syncthreads();
    const T off = s_excl + woff;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = wbase + j * kWave;
        if (i < n) wr(i, off + ex[j], it[j]);
    }
}

// Workspace of one scan over up to `cap` items (either schedule), bytes.
inline size_t scan_workspace(int64_t cap, int items = kScanItems) {
    const int64_t nb = scan_blocks(cap, items);
    return align_up(size_t(nb) * 8);
}

inline bool scan_one_pass(int64_t nb, bool sparse) { return sparse || nb <= kOnePassMaxBlocks; }

// Words at the start of the workspace that must be zero when a one-pass scan
// (the schedule taken when a status word is given) starts; 0 for the
// three-level schedule, which needs none.
inline int64_t scan_sync_words(int64_t cap, int items = kScanItems, bool sparse = false) {
    const int64_t nb = scan_blocks(cap, items);
    return scan_one_pass(nb, sparse) ? 2 * nb : 0;
}

// Scans up to `cap` items (the count read from d_n when given).  `ws` holds
// scan_workspace(cap, ITEMS) bytes; `d_status` (may be null) is also the word
// a bounded wait that expires reports into.  With `precleared` an earlier
// kernel of the stream zeroed the scan_sync_words(cap, ITEMS, sparse) words at
// `ws`.  `sparse`: the live count (d_n) is typically far below `cap`, so the
// one-pass schedule is taken at any capacity (its blocks past the live ones
// leave at once).
template <class T, int ITEMS = kScanItems, class Loader, class Writer>
void launch_scan(const Loader& ld, const Writer& wr, int64_t cap, const int64_t* d_n, const int32_t* d_status,
                 void* ws, T* total_out, hipStream_t stream, bool precleared = false, bool sparse = false) {
    const int64_t nb = scan_blocks(cap, ITEMS);
    char* base = static_cast<char*>(ws);
    if (scan_one_pass(nb, sparse) && d_status) {
        uint64_t* status = reinterpret_cast<uint64_t*>(base);
        if (!precleared) hipLaunchKernelGGL(k_scan_clear<256>, dim3(1), dim3(256), 0, stream, status, nb);
        hipLaunchKernelGGL((k_scan_onepass<T, ITEMS, Loader, Writer>), dim3(uint32_t(nb)), dim3(kScanThreads), 0, stream, ld,
                           wr, cap, d_n, d_status, status, total_out);
        return;
    }
    T* partials = reinterpret_cast<T*>(base);
    hipLaunchKernelGGL((k_scan_reduce<T, ITEMS, Loader>), dim3(uint32_t(nb)), dim3(kScanThreads), 0, stream, ld, cap, d_n,
                       d_status, partials);
    hipLaunchKernelGGL((k_scan_partials<T, ITEMS>), dim3(1), dim3(kPartialThreads), 0, stream, partials, nb, d_n, d_status,
                       total_out);
    hipLaunchKernelGGL((k_scan_down<T, ITEMS, Loader, Writer>), dim3(uint32_t(nb)), dim3(kScanThreads), 0, stream, ld, wr,
                       cap, d_n, d_status, partials);
}

}  // namespace ws
