// Stable LSD radix sort of (u64 key, u32 value) pairs (Sec. 3.3.2).
//
// Each pass places an element at base_d + prefix_wg + rank_local (Eq. 5-6):
//   base_d      count of the digits below d in the whole array,
//   prefix_wg   count of digit d in the tiles before this tile,
//   rank_local  rank among equal digits inside the tile, in input order,
//               which makes the sort stable.
// rank_local comes from wave64 ballots (a wave matches its lanes' digits bit
// by bit) and per-wave digit counters in LDS; the tile is reordered by digit
// in LDS so that global writes are runs of consecutive addresses.  A tile is
// 4096 pairs (256 threads x 16).
//
// Two schedules compute base_d + prefix_wg; they give identical bits:
//  * wait-free (large inputs): per pass, k_upsweep counts each tile's digits
//    into a digit-major table [digit][tile]; one exclusive scan of that table
//    (the hierarchical scan of scan.h, one dispatch per level) yields
//    base_d + prefix_wg for every (digit, tile) at once; k_downsweep ranks and
//    scatters.  No workgroup waits for another: this is the paper's
//    structure, with the table read as the "indicator stream" of all digits.
//  * look-back (small inputs, up to kLookbackMaxTiles tiles): base_d from one
//    histogram of all passes (k_sort_hist), prefix_wg by a decoupled look-back
//    over per-tile counts published in device memory.  Tiles take an atomic
//    ticket, so a tile only waits for tiles that have started, and the wait
//    is bounded (WS_ERR_SPIN_LIMIT on expiry).  One read and one write per
//    pair and pass, but the ticket serialises at about 12 ns per tile, which
//    is why large inputs use the wait-free schedule.
#include "scan.h"
#include "ws_internal.h"

namespace ws {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 pairs per tile
constexpr int kHistThreads = 256;
constexpr int kMaxBins = 2048;  // passes * radix over every radix width
constexpr int kLook = 16;       // predecessor tiles read at once by the look-back
constexpr int64_t kLookbackMaxTiles = 256;
constexpr uint32_t kStAgg = 1u << 30;
constexpr uint32_t kStInc = 2u << 30;
constexpr uint32_t kStMask = (1u << 30) - 1;

struct SortLayout {
    uint64_t* alt_keys;
    uint32_t* alt_vals;
    uint32_t* hist;      // look-back: [passes][radix]
    uint32_t* status;    // look-back: [passes][max_tiles][radix]
    uint32_t* tickets;   // look-back: [passes]
    uint32_t* table;     // wait-free: [radix][max_tiles]
    uint32_t* partials;  // wait-free: scan block sums of the table
    int64_t max_tiles;
    int passes, r, radix;
    bool wait_free;
};

int default_radix(int r) { return r <= 0 ? 8 : r; }

size_t plan(void* ws, int64_t capacity, int begin_bit, int end_bit, int radix_bits, SortLayout* out) {
    SortLayout L{};
    L.r = default_radix(radix_bits);
    L.radix = 1 << L.r;
    L.passes = (end_bit - begin_bit + L.r - 1) / L.r;
    L.max_tiles = std::max<int64_t>((capacity + kSortTile - 1) / kSortTile, 1);
    L.wait_free = L.max_tiles > kLookbackMaxTiles;
    char* base = static_cast<char*>(ws);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* ptr = base ? base + off : nullptr;
        off += align_up(bytes);
        return ptr;
    };
    if (L.passes > 1) {
        L.alt_keys = reinterpret_cast<uint64_t*>(take(size_t(capacity) * 8));
        L.alt_vals = reinterpret_cast<uint32_t*>(take(size_t(capacity) * 4));
    }
    if (L.wait_free) {
        const int64_t entries = int64_t(L.radix) * L.max_tiles;
        L.table = reinterpret_cast<uint32_t*>(take(size_t(entries) * 4));
        L.partials = reinterpret_cast<uint32_t*>(take(size_t(scan_blocks(entries)) * 4));
    } else {
        L.hist = reinterpret_cast<uint32_t*>(take(size_t(L.passes) * L.radix * 4));
        L.status = reinterpret_cast<uint32_t*>(take(size_t(L.passes) * L.max_tiles * L.radix * 4));
        L.tickets = reinterpret_cast<uint32_t*>(take(size_t(L.passes) * 4));
    }
    if (out) *out = L;
    return off;
}

__device__ __forceinline__ int64_t device_count(int64_t cap, const int64_t* d_n) {
    if (!d_n) return cap;
    const int64_t v = *d_n;
    return v < cap ? (v < 0 ? 0 : v) : cap;
}

// ------------------------------------------------------- tile ranking
//
// Loads tile `tile` (wave-striped: item j of lane l is element
// base + j*64 + l, so each wave's items are in input order) and computes, for
// every item, its rank among the equal digits of its wave.  On return
// s_whist[w][d] holds the exclusive prefix over waves of digit d's count and
// *cnt_out (threads t < RADIX) the tile's count of digit t.

template <int RADIX>
struct TileSmem {
    uint64_t keys[kSortTile];
    uint32_t vals[kSortTile];
    uint32_t whist[kSortWaves][RADIX];
    uint32_t tile_off[RADIX];
    uint32_t global[RADIX];
    uint32_t scan[kSortWaves + 1];
    uint32_t tile;
};

template <int R>
__device__ __forceinline__ void load_and_rank(TileSmem<1 << R>& sm, const uint64_t* kin, const uint32_t* vin,
                                              int64_t n, int64_t tile, int shift, int bits, uint64_t* key,
                                              uint32_t* val, uint32_t* rank, uint32_t* cnt_out) {
    constexpr int RADIX = 1 << R;
    const int wave = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const uint32_t dmask = (1u << bits) - 1u;
    const int64_t wbase = tile * kSortTile + int64_t(wave) * (kSortItems * kWave);
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int64_t idx = wbase + j * kWave + lane;
        const bool valid = idx < n;
        key[j] = valid ? kin[idx] : 0ull;
        val[j] = valid ? vin[idx] : 0u;
    }
    // Phase 1: lanes of the wave holding the same digit (matched bit by bit),
    // this lane's rank among them and the group's leader (lowest lane).
    // packed = below | leader << 8 | count << 16.
    uint32_t packed[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int64_t idx = wbase + j * kWave + lane;
        const bool valid = idx < n;
        const uint32_t d = uint32_t(key[j] >> shift) & dmask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t below = lanes_below(peers);
        const uint32_t leader = peers ? uint32_t(__builtin_ctzll(peers)) : 0u;
        const uint32_t cnt = (valid && below == 0) ? uint32_t(__popcll(peers)) : 0u;
        packed[j] = below | (leader << 8) | (cnt << 16);
    }
    // Phase 2: each group's leader adds the group size to the wave's digit
    // counter; LDS executes a wave's atomics in issue order, so item j sees the
    // counts of items 0..j-1 and the atomics need not wait for each other.
    uint32_t old[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const uint32_t cnt = packed[j] >> 16;
        const uint32_t d = uint32_t(key[j] >> shift) & dmask;
        old[j] = cnt ? atomicAdd(&sm.whist[wave][d], cnt) : 0u;
    }
    // Phase 3: every lane takes its group's base from the leader.
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const uint32_t leader = (packed[j] >> 8) & 0xffu;
        const uint32_t base = uint32_t(__shfl(int(old[j]), int(leader), kWave));
        rank[j] = base + (packed[j] & 0xffu);
    }
    __syncthreads();
    // per digit: exclusive prefix over the waves, and the tile's count
    const int t = threadIdx.x;
    uint32_t c = 0;
    if (t < RADIX) {
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            const uint32_t x = sm.whist[w][t];
            sm.whist[w][t] = c;
            c += x;
        }
    }
    *cnt_out = c;
}

// Reorders the ranked tile by digit in LDS and writes runs of equal digits
// to out positions global[d] + (position inside the digit's run).
template <int R>
__device__ __forceinline__ void scatter_tile(TileSmem<1 << R>& sm, int64_t n, int64_t tile, int shift, int bits,
                                             const uint64_t* key, const uint32_t* val, const uint32_t* rank,
                                             uint64_t* kout, uint32_t* vout) {
    const int wave = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const uint32_t dmask = (1u << bits) - 1u;
    const int64_t wbase = tile * kSortTile + int64_t(wave) * (kSortItems * kWave);
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int64_t idx = wbase + j * kWave + lane;
        if (idx < n) {
            const uint32_t d = uint32_t(key[j] >> shift) & dmask;
            const uint32_t pos = sm.tile_off[d] + sm.whist[wave][d] + rank[j];
            sm.keys[pos] = key[j];
            sm.vals[pos] = val[j];
        }
    }
    __syncthreads();
    const int tile_n = int(min<int64_t>(kSortTile, n - tile * kSortTile));
    for (int i = threadIdx.x; i < tile_n; i += kSortThreads) {
        const uint64_t k = sm.keys[i];
        const uint32_t d = uint32_t(k >> shift) & dmask;
        const uint32_t out = sm.global[d] + uint32_t(i) - sm.tile_off[d];
        if (int64_t(out) < n) {  // always true for consistent counts; guards the write
            kout[out] = k;
            vout[out] = sm.vals[i];
        }
    }
}

// ------------------------------------------------ wait-free schedule

struct UpArgs {
    const uint64_t* kin;
    int64_t cap;
    const int64_t* d_n;
    const int32_t* d_status;
    int shift, bits;
    uint32_t* table;
    int64_t max_tiles;
};

// Digit counts of one tile into table[d][tile] (zeros for tiles past the end).
template <int R>
__global__ __launch_bounds__(kSortThreads) void k_upsweep(UpArgs a) {
    constexpr int RADIX = 1 << R;
    __shared__ uint32_t s_h[kSortWaves][RADIX];
    if (a.d_status && *a.d_status != 0) return;
    const int64_t n = device_count(a.cap, a.d_n);
    const int64_t tile = blockIdx.x;
    const int wave = threadIdx.x / kWave;
    for (int i = threadIdx.x; i < kSortWaves * RADIX; i += kSortThreads) (&s_h[0][0])[i] = 0;
    __syncthreads();
    const uint32_t dmask = (1u << a.bits) - 1u;
    const int64_t base = tile * kSortTile;
    const uint32_t lane = lane_id();
#pragma unroll 4
    for (int j = 0; j < kSortItems; ++j) {
        const int64_t idx = base + int64_t(wave) * (kSortItems * kWave) + j * kWave + lane;
        const bool valid = idx < n;
        const uint32_t d = valid ? uint32_t(a.kin[idx] >> a.shift) & dmask : 0u;
        const uint64_t active = __ballot(valid);
        if (active == 0) continue;
        const uint32_t d0 = __builtin_amdgcn_readfirstlane(valid ? d : 0xffffffffu);
        // a wave whose valid lanes share one digit adds them with one atomic
        const uint64_t same = __ballot(valid && d == d0);
        if (same == active) {
            if (lanes_below(active) == 0 && valid) atomicAdd(&s_h[wave][d0], uint32_t(__popcll(active)));
        } else if (valid) {
            atomicAdd(&s_h[wave][d], 1u);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < RADIX; d += kSortThreads) {
        uint32_t s = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) s += s_h[w][d];
        a.table[int64_t(d) * a.max_tiles + tile] = s;
    }
}

struct DownArgs {
    const uint64_t* kin;
    const uint32_t* vin;
    uint64_t* kout;
    uint32_t* vout;
    int64_t cap;
    const int64_t* d_n;
    const int32_t* d_status;
    int shift, bits;
    const uint32_t* table;  // scanned: base_d + prefix_wg per (digit, tile)
    int64_t max_tiles;
};

template <int R>
__global__ __launch_bounds__(kSortThreads) void k_downsweep(DownArgs a) {
    constexpr int RADIX = 1 << R;
    __shared__ TileSmem<RADIX> sm;
    if (a.d_status && *a.d_status != 0) return;
    const int64_t n = device_count(a.cap, a.d_n);
    const int64_t tile = blockIdx.x;
    if (tile * kSortTile >= n) return;
    for (int i = threadIdx.x; i < kSortWaves * RADIX; i += kSortThreads) (&sm.whist[0][0])[i] = 0;
    __syncthreads();
    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t rank[kSortItems];
    uint32_t cnt;
    load_and_rank<R>(sm, a.kin, a.vin, n, tile, a.shift, a.bits, key, val, rank, &cnt);
    uint32_t total;
    const uint32_t toff = block_exclusive_scan<kSortThreads>(cnt, sm.scan, &total);
    if (threadIdx.x < RADIX) {
        sm.tile_off[threadIdx.x] = toff;
        sm.global[threadIdx.x] = a.table[int64_t(threadIdx.x) * a.max_tiles + tile];
    }
    __syncthreads();
    scatter_tile<R>(sm, n, tile, a.shift, a.bits, key, val, rank, a.kout, a.vout);
}

struct TableLoad {
    const uint32_t* t;
    __device__ uint32_t operator()(int64_t i) const { return t[i]; }
};
struct TableStore {
    uint32_t* t;
    __device__ void operator()(int64_t i, uint32_t prefix, uint32_t) const { t[i] = prefix; }
};

// ------------------------------------------------ look-back schedule

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
        const uint64_t active = __ballot(true);
        const bool first = lanes_below(active) == 0;
        for (int p = 0; p < a.passes; ++p) {
            const int sh = a.begin + p * a.r;
            const int nb = min(a.r, a.end - sh);
            const uint32_t d = uint32_t(k >> sh) & (mask_full >> (a.r - nb));
            const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
            const uint64_t same = __ballot(d == d0);
            if (same == active) {
                if (first) atomicAdd(&s_h[wave][p * radix + d0], uint32_t(__popcll(active)));
            } else {
                atomicAdd(&s_h[wave][p * radix + d], 1u);
            }
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
    __shared__ TileSmem<RADIX> sm;
    if (a.d_status && *a.d_status != 0) return;
    const int64_t n = device_count(a.cap, a.d_n);
    if (threadIdx.x == 0) sm.tile = atomicAdd(a.ticket, 1u);
    for (int i = threadIdx.x; i < kSortWaves * RADIX; i += kSortThreads) (&sm.whist[0][0])[i] = 0;
    __syncthreads();
    const int64_t tile = sm.tile;
    const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    if (tile >= ntiles) return;
    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t rank[kSortItems];
    uint32_t cnt;
    load_and_rank<R>(sm, a.kin, a.vin, n, tile, a.shift, a.bits, key, val, rank, &cnt);
    const int t = threadIdx.x;
    if (t < RADIX) store_agent(&a.status[tile * RADIX + t], (tile == 0 ? kStInc : kStAgg) | cnt);
    uint32_t total;
    const uint32_t toff = block_exclusive_scan<kSortThreads>(cnt, sm.scan, &total);
    const uint32_t hv = t < RADIX ? a.hist[t] : 0u;
    const uint32_t dbase = block_exclusive_scan<kSortThreads>(hv, sm.scan, &total);
    if (t < RADIX) {
        sm.tile_off[t] = toff;
        uint32_t excl = 0;
        if (tile > 0) {
            // Look back over windows of kLook predecessors with all loads in
            // flight: sum their counts, newest first, up to the first tile that
            // has published its inclusive prefix.  Tiles before tile 0 read as
            // an inclusive prefix of 0.
            int64_t k = tile - 1;
            uint32_t spins = 0;
            bool done = false;
            while (!done) {
                uint32_t s[kLook];
#pragma unroll
                for (int w = 0; w < kLook; ++w) s[w] = k - w >= 0 ? load_agent(&a.status[(k - w) * RADIX + t]) : kStInc;
                while (true) {
                    // usable once its prefix up to the first inclusive entry is published
                    bool blocked = false, seen_inc = false;
#pragma unroll
                    for (int w = 0; w < kLook; ++w) {
                        const uint32_t f = s[w] >> 30;
                        if (!seen_inc && !blocked) {
                            if (f == 0) blocked = true;
                            else if (f == 2) seen_inc = true;
                        }
                    }
                    if (!blocked) break;
                    if (++spins > kSpinLimit) {
                        if (a.d_status_rw) atomicExch(a.d_status_rw, int32_t(WS_ERR_SPIN_LIMIT));
                        done = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
#pragma unroll
                    for (int w = 0; w < kLook; ++w)
                        if ((s[w] >> 30) == 0) s[w] = load_agent(&a.status[(k - w) * RADIX + t]);
                }
                if (done) break;
#pragma unroll
                for (int w = 0; w < kLook; ++w) {
                    if (!done) {
                        excl += s[w] & kStMask;
                        if ((s[w] >> 30) == 2) done = true;
                    }
                }
                k -= kLook;
            }
            store_agent(&a.status[tile * RADIX + t], kStInc | (excl + cnt));
        }
        sm.global[t] = dbase + excl;
    }
    __syncthreads();
    scatter_tile<R>(sm, n, tile, a.shift, a.bits, key, val, rank, a.kout, a.vout);
}

template <int R>
void launch_pass_lookback(const PassArgs& pa, uint32_t grid, hipStream_t stream) {
    hipLaunchKernelGGL(k_sort_pass<R>, dim3(grid), dim3(kSortThreads), 0, stream, pa);
}

template <int R>
void launch_pass_wait_free(const UpArgs& ua, const DownArgs& da, uint32_t grid, uint32_t* partials,
                           const int32_t* d_status, hipStream_t stream) {
    hipLaunchKernelGGL(k_upsweep<R>, dim3(grid), dim3(kSortThreads), 0, stream, ua);
    const int64_t entries = int64_t(1 << R) * ua.max_tiles;
    launch_scan<uint32_t>(TableLoad{ua.table}, TableStore{ua.table}, entries, nullptr, d_status, partials,
                          static_cast<uint32_t*>(nullptr), stream);
    hipLaunchKernelGGL(k_downsweep<R>, dim3(grid), dim3(kSortThreads), 0, stream, da);
}

}  // namespace

size_t sort_workspace(int64_t capacity, int32_t begin_bit, int32_t end_bit, int32_t radix_bits) {
    return plan(nullptr, capacity, begin_bit, end_bit, radix_bits, nullptr);
}

hipError_t launch_sort(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout, int64_t n,
                       const int64_t* d_n, const int32_t* d_status, int32_t begin_bit, int32_t end_bit,
                       int32_t radix_bits, void* ws, hipStream_t stream, bool timed) {
    SortLayout L;
    plan(ws, n, begin_bit, end_bit, radix_bits, &L);
    const int hist_id = timed ? WS_KERNEL_SORT_HIST : -1, pass_id = timed ? WS_KERNEL_SORT_PASS : -1;
    const uint32_t grid = uint32_t(L.max_tiles);
    if (!L.wait_free) {
        hipLaunchKernelGGL(k_sort_init, dim3(1), dim3(256), 0, stream, L.hist, L.passes * L.radix, L.tickets,
                           L.passes);
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
        timing_begin(hist_id, stream);
        hipLaunchKernelGGL(k_sort_hist, dim3(uint32_t(hist_blocks)), dim3(kHistThreads), 0, stream, h);
        timing_end(hist_id, stream);
    }
    for (int p = 0; p < L.passes; ++p) {
        const uint64_t* pk = p == 0 ? kin : ((L.passes - p) % 2 == 0 ? kout : L.alt_keys);
        const uint32_t* pv = p == 0 ? vin : ((L.passes - p) % 2 == 0 ? vout : L.alt_vals);
        const bool to_out = (L.passes - 1 - p) % 2 == 0;
        uint64_t* ok = to_out ? kout : L.alt_keys;
        uint32_t* ov = to_out ? vout : L.alt_vals;
        const int shift = begin_bit + p * L.r;
        const int bits = std::min(L.r, end_bit - shift);
        timing_begin(pass_id, stream);
        if (L.wait_free) {
            UpArgs ua{pk, n, d_n, d_status, shift, bits, L.table, L.max_tiles};
            DownArgs da{pk, pv, ok, ov, n, d_n, d_status, shift, bits, L.table, L.max_tiles};
            switch (L.r) {
                case 1: launch_pass_wait_free<1>(ua, da, grid, L.partials, d_status, stream); break;
                case 2: launch_pass_wait_free<2>(ua, da, grid, L.partials, d_status, stream); break;
                case 3: launch_pass_wait_free<3>(ua, da, grid, L.partials, d_status, stream); break;
                case 4: launch_pass_wait_free<4>(ua, da, grid, L.partials, d_status, stream); break;
                case 5: launch_pass_wait_free<5>(ua, da, grid, L.partials, d_status, stream); break;
                case 6: launch_pass_wait_free<6>(ua, da, grid, L.partials, d_status, stream); break;
                case 7: launch_pass_wait_free<7>(ua, da, grid, L.partials, d_status, stream); break;
                default: launch_pass_wait_free<8>(ua, da, grid, L.partials, d_status, stream); break;
            }
        } else {
            PassArgs pa;
            pa.kin = pk;
            pa.vin = pv;
            pa.kout = ok;
            pa.vout = ov;
            pa.cap = n;
            pa.d_n = d_n;
            pa.d_status_rw = const_cast<int32_t*>(d_status);
            pa.d_status = d_status;
            pa.shift = shift;
            pa.bits = bits;
            pa.hist = L.hist + p * L.radix;
            pa.status = L.status + int64_t(p) * L.max_tiles * L.radix;
            pa.ticket = L.tickets + p;
            switch (L.r) {
                case 1: launch_pass_lookback<1>(pa, grid, stream); break;
                case 2: launch_pass_lookback<2>(pa, grid, stream); break;
                case 3: launch_pass_lookback<3>(pa, grid, stream); break;
                case 4: launch_pass_lookback<4>(pa, grid, stream); break;
                case 5: launch_pass_lookback<5>(pa, grid, stream); break;
                case 6: launch_pass_lookback<6>(pa, grid, stream); break;
                case 7: launch_pass_lookback<7>(pa, grid, stream); break;
                default: launch_pass_lookback<8>(pa, grid, stream); break;
            }
        }
        timing_end(pass_id, stream);
    }
    return hipGetLastError();
}

}  // namespace ws
