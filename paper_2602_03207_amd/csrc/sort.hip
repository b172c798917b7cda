// Stable LSD radix sort of (u64 key, u32 value) pairs (Sec. 3.3.2).
//
// Each pass places an element at base_d + prefix_wg + rank_local (Eq. 5-6):
//   base_d      exclusive sum over digits of the global digit histogram; all
//               passes' histograms come from ONE read of the keys (k_sort_hist);
//   prefix_wg   count of digit d in the tiles before this one, obtained by a
//               decoupled look-back over per-tile digit counts published in
//               device memory (tiles take an atomic ticket, so every tile a
//               workgroup waits for has already started; the wait is bounded
//               and reports WS_ERR_SPIN_LIMIT instead of hanging);
//   rank_local  rank among equal digits inside the tile, from wave64 ballots
//               (a wave matches its lanes' digits bit by bit) and per-wave
//               counters in LDS, in input order, which makes the sort stable.
// A pass reads 12 bytes and writes 12 bytes per pair; the tile is reordered
// by digit in LDS first so that the global writes are runs of consecutive
// addresses.  The paper's wait-free multi-dispatch scan is prior art; on
// MI355X the look-back keeps one read and one write per pair and pass.
#include "ws_internal.h"

namespace ws {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 pairs per tile
constexpr int kHistThreads = 256;
constexpr int kMaxBins = 2048;  // passes * radix over every radix width
constexpr uint32_t kStAgg = 1u << 30;
constexpr uint32_t kStInc = 2u << 30;
constexpr uint32_t kStMask = (1u << 30) - 1;

struct SortLayout {
    uint64_t* alt_keys;
    uint32_t* alt_vals;
    uint32_t* hist;     // [passes][radix]
    uint32_t* status;   // [passes][max_tiles][radix]
    uint32_t* tickets;  // [passes]
    int64_t max_tiles;
    int passes, r, radix;
};

int default_radix(int r) { return r <= 0 ? 8 : r; }

SortLayout plan(void* ws, int64_t capacity, int begin_bit, int end_bit, int radix_bits) {
    SortLayout L{};
    L.r = default_radix(radix_bits);
    L.radix = 1 << L.r;
    L.passes = (end_bit - begin_bit + L.r - 1) / L.r;
    L.max_tiles = std::max<int64_t>((capacity + kSortTile - 1) / kSortTile, 1);
    char* p = static_cast<char*>(ws);
    if (L.passes > 1) {
        L.alt_keys = reinterpret_cast<uint64_t*>(p);
        p += align_up(size_t(capacity) * 8);
        L.alt_vals = reinterpret_cast<uint32_t*>(p);
        p += align_up(size_t(capacity) * 4);
    }
    L.hist = reinterpret_cast<uint32_t*>(p);
    p += align_up(size_t(L.passes) * L.radix * 4);
    L.status = reinterpret_cast<uint32_t*>(p);
    p += align_up(size_t(L.passes) * L.max_tiles * L.radix * 4);
    L.tickets = reinterpret_cast<uint32_t*>(p);
    return L;
}

size_t plan_bytes(int64_t capacity, int begin_bit, int end_bit, int radix_bits) {
    const int r = default_radix(radix_bits);
    const int radix = 1 << r;
    const int passes = (end_bit - begin_bit + r - 1) / r;
    const int64_t max_tiles = std::max<int64_t>((capacity + kSortTile - 1) / kSortTile, 1);
    size_t b = 0;
    if (passes > 1) b += align_up(size_t(capacity) * 8) + align_up(size_t(capacity) * 4);
    b += align_up(size_t(passes) * radix * 4);
    b += align_up(size_t(passes) * max_tiles * radix * 4);
    b += align_up(size_t(passes) * 4);
    return b;
}

__device__ __forceinline__ int64_t device_count(int64_t cap, const int64_t* d_n) {
    if (!d_n) return cap;
    const int64_t v = *d_n;
    return v < cap ? (v < 0 ? 0 : v) : cap;
}

__global__ void k_sort_init(uint32_t* hist, int bins, uint32_t* tickets, int passes) {
    for (int i = threadIdx.x; i < bins; i += blockDim.x) hist[i] = 0;
    for (int i = threadIdx.x; i < passes; i += blockDim.x) tickets[i] = 0;
}

struct HistArgs {
    const uint64_t* keys;
    int64_t cap;
    const int64_t* d_n;
    const int32_t* d_status;
    int begin, end, r, passes;
    uint32_t* hist;
    uint32_t* status;
    int64_t max_tiles;
};

// Digit histograms of every pass from one read of the keys, and clearing of
// the look-back words of the tiles the passes will use.
__global__ __launch_bounds__(kHistThreads) void k_sort_hist(HistArgs a) {
    __shared__ uint32_t s_h[kHistThreads / kWave][kMaxBins];
    if (a.d_status && *a.d_status != 0) return;
    const int64_t n = device_count(a.cap, a.d_n);
    const int radix = 1 << a.r;
    const int bins = a.passes * radix;
    const int wave = threadIdx.x / kWave;
    for (int i = threadIdx.x; i < bins; i += kHistThreads) {
#pragma unroll
        for (int w = 0; w < kHistThreads / kWave; ++w) s_h[w][i] = 0;
    }
    // clear look-back words: [passes][tiles used][radix]
    const int64_t tiles = (n + kSortTile - 1) / kSortTile;
    const int64_t words = tiles * radix;
    const int64_t gsize = int64_t(gridDim.x) * kHistThreads;
    for (int p = 0; p < a.passes; ++p) {
        uint32_t* st = a.status + int64_t(p) * a.max_tiles * radix;
        for (int64_t i = int64_t(blockIdx.x) * kHistThreads + threadIdx.x; i < words; i += gsize) st[i] = 0;
    }
    __syncthreads();
    const uint32_t mask_full = uint32_t(radix - 1);
    for (int64_t i = int64_t(blockIdx.x) * kHistThreads + threadIdx.x; i < n; i += gsize) {
        const uint64_t k = a.keys[i];
        for (int p = 0; p < a.passes; ++p) {
            const int sh = a.begin + p * a.r;
            const int nb = min(a.r, a.end - sh);
            const uint32_t d = uint32_t(k >> sh) & (mask_full >> (a.r - nb));
            atomicAdd(&s_h[wave][p * radix + d], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < bins; i += kHistThreads) {
        uint32_t s = 0;
#pragma unroll
        for (int w = 0; w < kHistThreads / kWave; ++w) s += s_h[w][i];
        if (s) atomicAdd(&a.hist[i], s);
    }
}

struct PassArgs {
    const uint64_t* kin;
    const uint32_t* vin;
    uint64_t* kout;
    uint32_t* vout;
    int64_t cap;
    const int64_t* d_n;
    int32_t* d_status_rw;  // may be null
    const int32_t* d_status;
    int shift, bits;
    const uint32_t* hist;  // [radix] of this pass
    uint32_t* status;      // [max_tiles][radix] of this pass
    uint32_t* ticket;
};

template <int R>
__global__ __launch_bounds__(kSortThreads) void k_sort_pass(PassArgs a) {
    constexpr int RADIX = 1 << R;
    static_assert(RADIX <= kSortThreads, "one digit per thread");
    __shared__ uint64_t s_keys[kSortTile];
    __shared__ uint32_t s_vals[kSortTile];
    __shared__ uint32_t s_whist[kSortWaves][RADIX];
    __shared__ uint32_t s_tile_off[RADIX];
    __shared__ uint32_t s_global[RADIX];
    __shared__ uint32_t s_scan[kSortWaves + 1];
    __shared__ uint32_t s_tile;

    if (a.d_status && *a.d_status != 0) return;
    const int64_t n = device_count(a.cap, a.d_n);
    if (threadIdx.x == 0) s_tile = atomicAdd(a.ticket, 1u);
    const int wave = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    for (int i = threadIdx.x; i < kSortWaves * RADIX; i += kSortThreads) (&s_whist[0][0])[i] = 0;
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    if (tile >= ntiles) return;
    const uint32_t dmask = (1u << a.bits) - 1u;

    // ---- load (wave-striped: item j of lane l is element base + j*64 + l) and rank
    const int64_t wbase = tile * kSortTile + int64_t(wave) * (kSortItems * kWave);
    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t rank[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int64_t idx = wbase + j * kWave + lane;
        const bool valid = idx < n;
        key[j] = valid ? a.kin[idx] : 0ull;
        val[j] = valid ? a.vin[idx] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int64_t idx = wbase + j * kWave + lane;
        const bool valid = idx < n;
        const uint32_t d = uint32_t(key[j] >> a.shift) & dmask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < a.bits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t below = lanes_below(peers);
        const uint32_t base = s_whist[wave][d];
        rank[j] = base + below;
        __builtin_amdgcn_wave_barrier();
        if (valid && below == 0) s_whist[wave][d] = base + uint32_t(__popcll(peers));
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // ---- per digit: wave prefixes and the tile's count
    const int t = threadIdx.x;
    uint32_t cnt = 0;
    if (t < RADIX) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            const uint32_t c = s_whist[w][t];
            s_whist[w][t] = run;
            run += c;
        }
        cnt = run;
        store_agent(&a.status[tile * RADIX + t], (tile == 0 ? kStInc : kStAgg) | cnt);
    }
    uint32_t total;
    const uint32_t toff = block_exclusive_scan<kSortThreads>(cnt, s_scan, &total);
    const uint32_t hv = t < RADIX ? a.hist[t] : 0u;
    const uint32_t dbase = block_exclusive_scan<kSortThreads>(hv, s_scan, &total);
    if (t < RADIX) {
        s_tile_off[t] = toff;
        uint32_t excl = 0;
        if (tile > 0) {
            int64_t k = tile - 1;
            uint32_t spins = 0;
            while (k >= 0) {
                const uint32_t s = load_agent(&a.status[k * RADIX + t]);
                if ((s >> 30) == 0) {
                    if (++spins > kSpinLimit) {
                        if (a.d_status_rw) atomicExch(a.d_status_rw, int32_t(WS_ERR_SPIN_LIMIT));
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += s & kStMask;
                if ((s >> 30) == 2) break;
                --k;
            }
            store_agent(&a.status[tile * RADIX + t], kStInc | (excl + cnt));
        }
        s_global[t] = dbase + excl;
    }
    __syncthreads();

    // ---- reorder the tile by digit in LDS
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int64_t idx = wbase + j * kWave + lane;
        if (idx < n) {
            const uint32_t d = uint32_t(key[j] >> a.shift) & dmask;
            const uint32_t pos = s_tile_off[d] + s_whist[wave][d] + rank[j];
            s_keys[pos] = key[j];
            s_vals[pos] = val[j];
        }
    }
    __syncthreads();

    // ---- write runs of equal digits to their global positions
    const int tile_n = int(min<int64_t>(kSortTile, n - tile * kSortTile));
    for (int i = threadIdx.x; i < tile_n; i += kSortThreads) {
        const uint64_t k = s_keys[i];
        const uint32_t d = uint32_t(k >> a.shift) & dmask;
        const uint32_t out = s_global[d] + uint32_t(i) - s_tile_off[d];
        if (int64_t(out) < n) {  // always true for a consistent histogram; guards the write
            a.kout[out] = k;
            a.vout[out] = s_vals[i];
        }
    }
}

template <int R>
void launch_pass(const PassArgs& pa, uint32_t grid, hipStream_t stream) {
    hipLaunchKernelGGL(k_sort_pass<R>, dim3(grid), dim3(kSortThreads), 0, stream, pa);
}

}  // namespace

size_t sort_workspace(int64_t capacity, int32_t begin_bit, int32_t end_bit, int32_t radix_bits) {
    return plan_bytes(capacity, begin_bit, end_bit, radix_bits);
}

hipError_t launch_sort(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout, int64_t n,
                       const int64_t* d_n, const int32_t* d_status, int32_t begin_bit, int32_t end_bit,
                       int32_t radix_bits, void* ws, hipStream_t stream) {
    SortLayout L = plan(ws, n, begin_bit, end_bit, radix_bits);
    hipLaunchKernelGGL(k_sort_init, dim3(1), dim3(256), 0, stream, L.hist, L.passes * L.radix, L.tickets, L.passes);
    HistArgs h;
    h.keys = kin;
    h.cap = n;
    h.d_n = d_n;
    h.d_status = d_status;
    h.begin = begin_bit;
    h.end = end_bit;
    h.r = L.r;
    h.passes = L.passes;
    h.hist = L.hist;
    h.status = L.status;
    h.max_tiles = L.max_tiles;
    const int64_t hist_blocks = std::min<int64_t>(std::max<int64_t>((n + 4095) / 4096, 1), 2048);
    timing_begin(WS_KERNEL_SORT_HIST, stream);
    hipLaunchKernelGGL(k_sort_hist, dim3(uint32_t(hist_blocks)), dim3(kHistThreads), 0, stream, h);
    timing_end(WS_KERNEL_SORT_HIST, stream);
    const uint32_t grid = uint32_t(L.max_tiles);
    for (int p = 0; p < L.passes; ++p) {
        PassArgs pa;
        pa.kin = p == 0 ? kin : ((L.passes - p) % 2 == 0 ? kout : L.alt_keys);
        pa.vin = p == 0 ? vin : ((L.passes - p) % 2 == 0 ? vout : L.alt_vals);
        const bool to_out = (L.passes - 1 - p) % 2 == 0;
        pa.kout = to_out ? kout : L.alt_keys;
        pa.vout = to_out ? vout : L.alt_vals;
        pa.cap = n;
        pa.d_n = d_n;
        pa.d_status_rw = const_cast<int32_t*>(d_status);
        pa.d_status = d_status;
        pa.shift = begin_bit + p * L.r;
        pa.bits = std::min(L.r, end_bit - pa.shift);
        pa.hist = L.hist + p * L.radix;
        pa.status = L.status + int64_t(p) * L.max_tiles * L.radix;
        pa.ticket = L.tickets + p;
        timing_begin(WS_KERNEL_SORT_PASS, stream);
        switch (L.r) {
            case 1: launch_pass<1>(pa, grid, stream); break;
            case 2: launch_pass<2>(pa, grid, stream); break;
            case 3: launch_pass<3>(pa, grid, stream); break;
            case 4: launch_pass<4>(pa, grid, stream); break;
            case 5: launch_pass<5>(pa, grid, stream); break;
            case 6: launch_pass<6>(pa, grid, stream); break;
            case 7: launch_pass<7>(pa, grid, stream); break;
            default: launch_pass<8>(pa, grid, stream); break;
        }
        timing_end(WS_KERNEL_SORT_PASS, stream);
    }
    return hipGetLastError();
}

}  // namespace ws
