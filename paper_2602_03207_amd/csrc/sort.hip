// Stable LSD radix sort of (key, u32 value) pairs, keys of 64 or 32 bits
// (Sec. 3.3.2).
//
// Each pass places an element at base_d + prefix_wg + rank_local (Eq. 5-6):
//   base_d      count of the digits below d in the whole array,
//   prefix_wg   count of digit d in the tiles before this tile,
//   rank_local  rank among equal digits inside the tile, in input order,
//               which makes the sort stable.
// rank_local comes from wave64 ballots (a wave matches its lanes' digits bit
// by bit, the bit count of the pass fixed at compile time) and per-wave digit
// counters in LDS; the tile is reordered by digit in LDS, keys first and then
// values through the same buffer, so that global writes are runs of
// consecutive addresses.  A tile is 256 threads x ITEMS pairs: 4096 pairs for
// large inputs, 2048 for mid-sized ones and 1024 for small ones, so that they
// still spread over the CUs.
//
// Two schedules compute base_d + prefix_wg; they give identical bits:
//  * look-back (small inputs, up to kSmallSortMax pairs, or inputs whose
//    device count is known to be far below the capacity): base_d from one
//    histogram of all passes (k_sort_hist), prefix_wg by a decoupled look-back
//    over per-tile counts published in device memory.  Workgroup b sorts tile
//    b, and the grid covers every tile the capacity can hold (workgroups past
//    the live tiles leave at once).  A tile waits only for tiles with smaller
//    indices, and the smallest unfinished tile is always running: each XCD
//    starts its workgroups in index order, so its resources can only be held
//    by tiles with smaller indices, which have finished.  The wait is bounded
//    (WS_ERR_SPIN_LIMIT on expiry).  One read and one write per pair and pass,
//    and one launch per pass.
//  * wait-free (large inputs, where the look-back chain in front of every
//    tile's writes and the histogram's extra read cost more than they save):
//    per pass, k_upsweep counts each tile's digits into a digit-major table
//    [digit][tile]; one exclusive scan of that table (the hierarchical scan of
//    scan.h) yields base_d + prefix_wg for every (digit, tile) at once;
//    k_downsweep ranks and scatters.  No workgroup waits for another.  Tiles
//    are laid out XCD-contiguously, so the table's entries of neighbouring
//    tiles, and the partly written lines where their digit runs meet, stay in
//    one L2.
#include "scan.h"
#include "ws_internal.h"

namespace ws {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kItemsLarge = 16;              // 4096-pair tiles
constexpr int kItemsMid = 8;                 // 2048-pair tiles
constexpr int kItemsSmall = 4;               // 1024-pair tiles
constexpr int64_t kSmallSortMax = 1 << 20;   // capacities up to this use small tiles
constexpr int64_t kMidSortMax = 1 << 23;     // wait-free sorts up to this use 2048-pair tiles
constexpr int kHistThreads = 256;
constexpr int kMaxBins = 2048;  // passes * radix of the look-back schedule's histograms, at most
constexpr int kLook = 16;       // predecessor tiles read at once by the look-back
constexpr int kTableItems = 4;  // items per thread of the digit table's prefix sum
constexpr uint32_t kStAgg = 1u << 30;
constexpr uint32_t kStInc = 2u << 30;
constexpr uint32_t kStMask = (1u << 30) - 1;

struct SortLayout {
    void* alt_keys;      // [capacity] keys of the key width
    uint32_t* alt_vals;
    uint32_t* hist;      // look-back: [passes][radix]
    uint32_t* status;    // look-back: [passes][max_tiles][radix]
    uint32_t* table;     // wait-free: [radix][max_tiles]
    void* table_scan;    // wait-free: workspace of the table's prefix sum
    int64_t max_tiles;
    int passes, r, radix, items;
    bool wait_free;
};

int default_radix(int r) { return r <= 0 ? 8 : r; }

size_t plan(void* ws, int64_t capacity, int begin_bit, int end_bit, int radix_bits, bool sparse, int key_bytes,
            SortLayout* out) {
    SortLayout L{};
    L.r = default_radix(radix_bits);
    L.radix = 1 << L.r;
    L.passes = (end_bit - begin_bit + L.r - 1) / L.r;
    const bool small = sparse || capacity <= kSmallSortMax;
    // the look-back schedule's histograms of all passes fit kMaxBins: a wider
    // digit than that allows is narrowed (the order is the same at any width)
    while (small && L.r > 1 && L.passes * L.radix > kMaxBins) {
        --L.r;
        L.radix = 1 << L.r;
        L.passes = (end_bit - begin_bit + L.r - 1) / L.r;
    }
    // wait-free tiles: 2048 pairs up to 8 M pairs of capacity (twice the
    // workgroups of 4096-pair tiles for a 1080p frame's 1-2 M pairs), 4096
    // above, where longer digit runs make the scatter's writes whole lines
    L.items = small ? kItemsSmall : (capacity <= kMidSortMax ? kItemsMid : kItemsLarge);
    const int64_t tile = int64_t(kSortThreads) * L.items;
    L.max_tiles = std::max<int64_t>((capacity + tile - 1) / tile, 1);
    L.wait_free = !small;
    char* base = static_cast<char*>(ws);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* ptr = base ? base + off : nullptr;
        off += align_up(bytes);
        return ptr;
    };
    if (L.passes > 1) {
        L.alt_keys = take(size_t(capacity) * size_t(key_bytes));
        L.alt_vals = reinterpret_cast<uint32_t*>(take(size_t(capacity) * 4));
    }
    if (L.wait_free) {
        const int64_t entries = int64_t(L.radix) * L.max_tiles;
        L.table = reinterpret_cast<uint32_t*>(take(size_t(entries) * 4));
        L.table_scan = take(scan_workspace(entries, kTableItems));
    } else {
        L.hist = reinterpret_cast<uint32_t*>(take(size_t(L.passes) * L.radix * 4));
        L.status = reinterpret_cast<uint32_t*>(take(size_t(L.passes) * L.max_tiles * L.radix * 4));
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
// B: digit bits of the pass; ITEMS: pairs per thread.  Item j of lane l in
// wave w is element tile*TILE + w*ITEMS*64 + j*64 + l, so each wave's items
// are in input order.

template <int B, int ITEMS, typename K>
struct TileSmem {
    static constexpr int kTile = kSortThreads * ITEMS;
    static constexpr int kRadix = 1 << B;
    K buf[kTile];  // reorder buffer: keys, then values (as u32)
    uint32_t whist[kSortWaves][kRadix];
    uint32_t tile_off[kRadix];
    uint32_t global[kRadix];
    uint32_t scan[kSortWaves + 1];
};

template <int B, typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift) {
    return uint32_t(k >> shift) & ((1u << B) - 1u);
}

// Per-digit work is spread over the workgroup in blocks: thread t owns digits
// t * DPT ... t * DPT + DPT - 1 (DPT = 1 up to 8-bit digits, where threads
// t >= 2^B own none), so a thread's digits are consecutive in digit order.
template <int B>
constexpr int digits_per_thread() {
    return (1 << B) > kSortThreads ? (1 << B) / kSortThreads : 1;
}

// Exclusive prefix over digit order of per-digit values held DPT per thread.
template <int DPT>
__device__ __forceinline__ void digit_exclusive_scan(const uint32_t (&v)[DPT], uint32_t (&ex)[DPT], uint32_t* scratch) {
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
        ex[i] = s;
        s += v[i];
    }
    uint32_t total;
    const uint32_t base = block_exclusive_scan<kSortThreads>(s, scratch, &total);
#pragma unroll
    for (int i = 0; i < DPT; ++i) ex[i] += base;
}

// Loads the tile and computes, for every item, its rank among the equal
// digits of its wave.  On return whist[w][d] holds the exclusive prefix over
// waves of digit d's count and cnt_out[i] the tile's count of this thread's
// digit i (zero for digits past 2^B).  whist must be zero on entry.
template <int B, int ITEMS, typename K>
__device__ __forceinline__ void load_and_rank(TileSmem<B, ITEMS, K>& sm, const K* kin, int64_t n, int64_t tile,
                                              int shift, K* key, uint32_t* rank,
                                              uint32_t (&cnt_out)[digits_per_thread<B>()]) {
    constexpr int kTile = kSortThreads * ITEMS;
    const int wave = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const int64_t wbase = tile * kTile + int64_t(wave) * (ITEMS * kWave);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t idx = wbase + j * kWave + lane;
        key[j] = idx < n ? kin[idx] : K(0);
    }
    // Phase 1: lanes of the wave holding the same digit (matched bit by bit),
    // this lane's rank among them and the group's leader (lowest lane).
    // packed = below | leader << 8 | count << 16.
    uint32_t packed[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const bool valid = wbase + j * kWave + lane < n;
        const uint32_t d = digit_of<B>(key[j], shift);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < B; ++b) {
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
    uint32_t old[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t cnt = packed[j] >> 16;
        old[j] = cnt ? atomicAdd(&sm.whist[wave][digit_of<B>(key[j], shift)], cnt) : 0u;
    }
    // Phase 3: every lane takes its group's base from the leader.
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t leader = (packed[j] >> 8) & 0xffu;
        const uint32_t base = uint32_t(__shfl(int(old[j]), int(leader), kWave));
        rank[j] = base + (packed[j] & 0xffu);
    }
    __syncthreads();
    // per digit: exclusive prefix over the waves, and the tile's count
    constexpr int DPT = digits_per_thread<B>();
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
        const int d = int(threadIdx.x) * DPT + i;
        uint32_t c = 0;
        if (d < (1 << B)) {
#pragma unroll
            for (int w = 0; w < kSortWaves; ++w) {
                const uint32_t x = sm.whist[w][d];
                sm.whist[w][d] = c;
                c += x;
            }
        }
        cnt_out[i] = c;
    }
}

// Reordering of a ranked tile by digit through LDS, so that global writes are
// runs of consecutive addresses: stage_keys puts each key at its position in
// the reordered tile (rank becomes that position), flush_tile writes runs of
// equal digits to global[d] + (position inside the digit's run), keys first
// and values second through the same buffer.  The values are read only after
// the keys are staged, which keeps them out of registers during the ranking.
// Requires tile_off (and for flush_tile global) visible to the workgroup.
template <int B, int ITEMS, typename K>
__device__ __forceinline__ void stage_keys(TileSmem<B, ITEMS, K>& sm, int64_t n, int64_t tile, int shift,
                                           const K* key, uint32_t* rank) {
    constexpr int kTile = kSortThreads * ITEMS;
    const int wave = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const int64_t wbase = tile * kTile + int64_t(wave) * (ITEMS * kWave);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t d = digit_of<B>(key[j], shift);
        rank[j] += sm.tile_off[d] + sm.whist[wave][d];
        if (wbase + j * kWave + lane < n) sm.buf[rank[j]] = key[j];
    }
}

template <int ITEMS>
__device__ __forceinline__ void load_vals(const uint32_t* vin, int64_t n, int64_t tile, uint32_t* val) {
    constexpr int kTile = kSortThreads * ITEMS;
    const int64_t wbase = tile * kTile + int64_t(threadIdx.x / kWave) * (ITEMS * kWave);
    const uint32_t lane = lane_id();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t idx = wbase + j * kWave + lane;
        val[j] = idx < n ? vin[idx] : 0u;
    }
}

// Caller synchronises the workgroup between stage_keys and this call.
template <int B, int ITEMS, typename K>
__device__ __forceinline__ void flush_tile(TileSmem<B, ITEMS, K>& sm, int64_t n, int64_t tile, int shift,
                                           const uint32_t* pos, const uint32_t* val, K* kout, uint32_t* vout) {
    constexpr int kTile = kSortThreads * ITEMS;
    const int wave = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const int64_t wbase = tile * kTile + int64_t(wave) * (ITEMS * kWave);
    const int tile_n = int(min<int64_t>(kTile, n - tile * kTile));
    uint32_t out[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int i = threadIdx.x + k * kSortThreads;
        out[k] = 0xffffffffu;
        if (i < tile_n) {
            const K kk = sm.buf[i];
            const uint32_t d = digit_of<B>(kk, shift);
            out[k] = sm.global[d] + uint32_t(i) - sm.tile_off[d];
            if (int64_t(out[k]) < n) kout[out[k]] = kk;  // always true for consistent counts; guards the write
        }
    }
    __syncthreads();
    uint32_t* vbuf = reinterpret_cast<uint32_t*>(sm.buf);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
        if (wbase + j * kWave + lane < n) vbuf[pos[j]] = val[j];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int i = threadIdx.x + k * kSortThreads;
        if (i < tile_n && int64_t(out[k]) < n) vout[out[k]] = vbuf[i];
    }
}

template <int B, int ITEMS, typename K>
__device__ __forceinline__ void clear_whist(TileSmem<B, ITEMS, K>& sm) {
    for (int i = threadIdx.x; i < kSortWaves * (1 << B); i += kSortThreads) (&sm.whist[0][0])[i] = 0;
}

// ------------------------------------------------ wait-free schedule

template <typename K>
struct UpArgs {
    const K* kin;
    int64_t cap;
    const int64_t* d_n;
    const int32_t* d_status;
    int shift;
    uint32_t* table;
    int64_t max_tiles;
    uint32_t* clear;  // look-back words of the table's prefix sum, zeroed here
    int64_t clear_words;
};

// Digit counts of one tile into table[d][tile] (zeros for tiles past the end).
template <int B, int ITEMS, typename K>
__global__ __launch_bounds__(kSortThreads) void k_upsweep(UpArgs<K> a) {
    constexpr int RADIX = 1 << B;
    constexpr int kTile = kSortThreads * ITEMS;
    __shared__ uint32_t s_h[kSortWaves][RADIX];
    for (int64_t i = int64_t(blockIdx.x) * kSortThreads + threadIdx.x; i < a.clear_words;
         i += int64_t(gridDim.x) * kSortThreads)
        a.clear[i] = 0u;
    if (a.d_status && *a.d_status != 0) return;
    const int64_t n = device_count(a.cap, a.d_n);
    const int64_t ntiles = (n + kTile - 1) / kTile;
    // live tiles in XCD-contiguous order; the others write their zero counts
    const int64_t tile = int64_t(blockIdx.x) < ntiles ? int64_t(xcd_contiguous(blockIdx.x, uint32_t(ntiles)))
                                                       : int64_t(blockIdx.x);
    const int wave = threadIdx.x / kWave;
    for (int i = threadIdx.x; i < kSortWaves * RADIX; i += kSortThreads) (&s_h[0][0])[i] = 0;
    __syncthreads();
    const int64_t wbase = tile * kTile + int64_t(wave) * (ITEMS * kWave) + lane_id();
    // all of the tile's loads in flight before the first use
    K k[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t idx = wbase + j * kWave;
        k[j] = idx < n ? a.kin[idx] : K(0);
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const bool valid = wbase + j * kWave < n;
        const uint32_t d = digit_of<B>(k[j], a.shift);
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

template <typename K>
struct DownArgs {
    const K* kin;
    const uint32_t* vin;
    K* kout;
    uint32_t* vout;
    int64_t cap;
    const int64_t* d_n;
    const int32_t* d_status;
    int shift;
    const uint32_t* table;  // scanned: base_d + prefix_wg per (digit, tile)
    int64_t max_tiles;
};

template <int B, int ITEMS, typename K>
__global__ __launch_bounds__(kSortThreads) void k_downsweep(DownArgs<K> a) {
    constexpr int kTile = kSortThreads * ITEMS;
    __shared__ TileSmem<B, ITEMS, K> sm;
    if (a.d_status && *a.d_status != 0) return;
    const int64_t n = device_count(a.cap, a.d_n);
    const int64_t ntiles = (n + kTile - 1) / kTile;
    if (int64_t(blockIdx.x) >= ntiles) return;
    const int64_t tile = xcd_contiguous(blockIdx.x, uint32_t(ntiles));
    clear_whist(sm);
    __syncthreads();
    constexpr int DPT = digits_per_thread<B>();
    K key[ITEMS];
    uint32_t rank[ITEMS];
    uint32_t cnt[DPT];
    load_and_rank<B, ITEMS, K>(sm, a.kin, n, tile, a.shift, key, rank, cnt);
    // the values are in flight during the scan and the staging of the keys
    uint32_t val[ITEMS];
    load_vals<ITEMS>(a.vin, n, tile, val);
    uint32_t toff[DPT];
    digit_exclusive_scan<DPT>(cnt, toff, sm.scan);
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
        const int d = int(threadIdx.x) * DPT + i;
        if (d < (1 << B)) {
            sm.tile_off[d] = toff[i];
            sm.global[d] = a.table[int64_t(d) * a.max_tiles + tile];
        }
    }
    __syncthreads();
    stage_keys<B, ITEMS, K>(sm, n, tile, a.shift, key, rank);
    __syncthreads();
    flush_tile<B, ITEMS, K>(sm, n, tile, a.shift, rank, val, a.kout, a.vout);
}

struct TableLoad {
    using Item = uint32_t;
    const uint32_t* t;
    __device__ uint32_t operator()(int64_t i) const { return t[i]; }
    __device__ static uint32_t value(uint32_t c) { return c; }
};
struct TableStore {
    uint32_t* t;
    __device__ void operator()(int64_t i, uint32_t prefix, uint32_t) const { t[i] = prefix; }
};

// ------------------------------------------------ look-back schedule

__global__ void k_sort_init(uint32_t* hist, int bins) {
    for (int i = threadIdx.x; i < bins; i += blockDim.x) hist[i] = 0;
}

template <typename K>
struct HistArgs {
    const K* keys;
    int64_t cap;
    const int64_t* d_n;
    const int32_t* d_status;
    int begin, end, r, passes;
    int tile;  // pairs per sort tile
    uint32_t* hist;
    uint32_t* status;
    int64_t max_tiles;
};

// Digit histograms of every pass from one read of the keys, and clearing of
// the look-back words of the tiles the passes will use.
template <typename K>
__global__ __launch_bounds__(kHistThreads) void k_sort_hist(HistArgs<K> a) {
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
    const int64_t tiles = (n + a.tile - 1) / a.tile;
    const int64_t words = tiles * radix;
    const int64_t gsize = int64_t(gridDim.x) * kHistThreads;
    for (int p = 0; p < a.passes; ++p) {
        uint32_t* st = a.status + int64_t(p) * a.max_tiles * radix;
        for (int64_t i = int64_t(blockIdx.x) * kHistThreads + threadIdx.x; i < words; i += gsize) st[i] = 0;
    }
    __syncthreads();
    const uint32_t mask_full = uint32_t(radix - 1);
    for (int64_t i = int64_t(blockIdx.x) * kHistThreads + threadIdx.x; i < n; i += gsize) {
        const K k = a.keys[i];
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

template <typename K>
struct PassArgs {
    const K* kin;
    const uint32_t* vin;
    K* kout;
    uint32_t* vout;
    int64_t cap;
    const int64_t* d_n;
    int32_t* d_status_rw;  // may be null
    const int32_t* d_status;
    int shift;
    const uint32_t* hist;  // [radix] of this pass
    uint32_t* status;      // [max_tiles][2^B] of this pass
};

template <int B, int ITEMS, typename K>
__device__ __forceinline__ void sort_tile_lookback(TileSmem<B, ITEMS, K>& sm, const PassArgs<K>& a, int64_t n,
                                                   int64_t tile) {
    constexpr int RADIX = 1 << B;
    constexpr int DPT = digits_per_thread<B>();
    K key[ITEMS];
    uint32_t rank[ITEMS];
    uint32_t cnt[DPT];
    load_and_rank<B, ITEMS, K>(sm, a.kin, n, tile, a.shift, key, rank, cnt);
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
        const int d = int(threadIdx.x) * DPT + i;
        if (d < RADIX) store_agent(&a.status[tile * RADIX + d], (tile == 0 ? kStInc : kStAgg) | cnt[i]);
    }
    uint32_t toff[DPT], hv[DPT], dbase[DPT];
    digit_exclusive_scan<DPT>(cnt, toff, sm.scan);
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
        const int d = int(threadIdx.x) * DPT + i;
        hv[i] = d < RADIX ? a.hist[d] : 0u;
    }
    digit_exclusive_scan<DPT>(hv, dbase, sm.scan);
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
        const int d = int(threadIdx.x) * DPT + i;
        if (d < RADIX) sm.tile_off[d] = toff[i];
    }
    __syncthreads();
    // the keys wait in LDS (and the values are in flight) during the look-back
    stage_keys<B, ITEMS, K>(sm, n, tile, a.shift, key, rank);
    uint32_t val[ITEMS];
    load_vals<ITEMS>(a.vin, n, tile, val);
    for (int i = 0; i < DPT; ++i) {
        const int t = int(threadIdx.x) * DPT + i;  // the digit
        if (t >= RADIX) break;
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
            store_agent(&a.status[tile * RADIX + t], kStInc | (excl + cnt[i]));
        }
        sm.global[t] = dbase[i] + excl;
    }
    __syncthreads();
    flush_tile<B, ITEMS, K>(sm, n, tile, a.shift, rank, val, a.kout, a.vout);
}

template <int B, int ITEMS, typename K>
__global__ __launch_bounds__(kSortThreads) void k_sort_pass(PassArgs<K> a) {
    constexpr int kTile = kSortThreads * ITEMS;
    __shared__ TileSmem<B, ITEMS, K> sm;
    if (a.d_status && *a.d_status != 0) return;
    const int64_t n = device_count(a.cap, a.d_n);
    const int64_t ntiles = (n + kTile - 1) / kTile;
    // Workgroups past the live tiles leave at once; workgroup b sorts tile b.
    if (int64_t(blockIdx.x) >= ntiles) return;
    clear_whist(sm);
    __syncthreads();
    sort_tile_lookback<B, ITEMS, K>(sm, a, n, int64_t(blockIdx.x));
}

// ------------------------------------------------ dispatch

template <typename K>
struct PassLaunch {
    const SortLayout* L;
    UpArgs<K> ua;
    DownArgs<K> da;
    PassArgs<K> pa;
    const int32_t* d_status;
    hipStream_t stream;
};

template <int B, int ITEMS, typename K>
void run_pass(const PassLaunch<K>& c) {
    const uint32_t grid = uint32_t(c.L->max_tiles);
    if (c.L->wait_free) {
        hipLaunchKernelGGL((k_upsweep<B, ITEMS, K>), dim3(grid), dim3(kSortThreads), 0, c.stream, c.ua);
        // the upsweep zeroed the scan's look-back words (c.ua.clear)
        const int64_t entries = int64_t(1 << B) * c.L->max_tiles;
        launch_scan<uint32_t, kTableItems>(TableLoad{c.ua.table}, TableStore{c.ua.table}, entries, nullptr, c.d_status,
                              c.L->table_scan, static_cast<uint32_t*>(nullptr), c.stream, true);
        hipLaunchKernelGGL((k_downsweep<B, ITEMS, K>), dim3(grid), dim3(kSortThreads), 0, c.stream, c.da);
    } else {
        hipLaunchKernelGGL((k_sort_pass<B, ITEMS, K>), dim3(grid), dim3(kSortThreads), 0, c.stream, c.pa);
    }
}

template <int ITEMS, typename K>
void run_pass_bits(const PassLaunch<K>& c, int bits) {
    switch (bits) {
        case 1: run_pass<1, ITEMS, K>(c); break;
        case 2: run_pass<2, ITEMS, K>(c); break;
        case 3: run_pass<3, ITEMS, K>(c); break;
        case 4: run_pass<4, ITEMS, K>(c); break;
        case 5: run_pass<5, ITEMS, K>(c); break;
        case 6: run_pass<6, ITEMS, K>(c); break;
        case 7: run_pass<7, ITEMS, K>(c); break;
        case 8: run_pass<8, ITEMS, K>(c); break;
        case 9: run_pass<9, ITEMS, K>(c); break;
        default: run_pass<10, ITEMS, K>(c); break;
    }
}

}  // namespace

size_t sort_workspace(int64_t capacity, int32_t begin_bit, int32_t end_bit, int32_t radix_bits, bool sparse,
                      int key_bytes) {
    return plan(nullptr, capacity, begin_bit, end_bit, radix_bits, sparse, key_bytes, nullptr);
}

void sort_sync_words(void* ws, int64_t capacity, int32_t begin_bit, int32_t end_bit, int32_t radix_bits, bool sparse,
                     int key_bytes, ClearList* c) {
    SortLayout L;
    plan(ws, capacity, begin_bit, end_bit, radix_bits, sparse, key_bytes, &L);
    if (!L.wait_free) c->add(L.hist, int64_t(L.passes) * L.radix);
}

SortHistWords sort_hist_words(void* ws, int64_t capacity, int32_t begin_bit, int32_t end_bit, int32_t radix_bits,
                              bool sparse, int key_bytes) {
    SortLayout L;
    plan(ws, capacity, begin_bit, end_bit, radix_bits, sparse, key_bytes, &L);
    SortHistWords w{};
    if (L.wait_free) return w;
    w.hist = L.hist;
    w.status = L.status;
    w.max_tiles = L.max_tiles;
    w.passes = L.passes;
    w.radix = L.radix;
    w.r = L.r;
    w.tile = kSortThreads * L.items;
    return w;
}

namespace {

template <typename K>
hipError_t launch_sort_t(const K* kin, const uint32_t* vin, K* kout, uint32_t* vout, int64_t n, const int64_t* d_n,
                         const int32_t* d_status, int32_t begin_bit, int32_t end_bit, int32_t radix_bits, void* ws,
                         hipStream_t stream, bool timed, bool sparse, bool precleared, bool hist_ready) {
    SortLayout L;
    plan(ws, n, begin_bit, end_bit, radix_bits, sparse, int(sizeof(K)), &L);
    K* alt_keys = static_cast<K*>(L.alt_keys);
    const int hist_id = timed ? WS_KERNEL_SORT_HIST : -1, pass_id = timed ? WS_KERNEL_SORT_PASS : -1;
    if (!L.wait_free && !hist_ready) {
        if (!precleared)
            hipLaunchKernelGGL(k_sort_init, dim3(1), dim3(256), 0, stream, L.hist, L.passes * L.radix);
        HistArgs<K> h;
        h.keys = kin;
        h.cap = n;
        h.d_n = d_n;
        h.d_status = d_status;
        h.begin = begin_bit;
        h.end = end_bit;
        h.r = L.r;
        h.passes = L.passes;
        h.tile = kSortThreads * L.items;
        h.hist = L.hist;
        h.status = L.status;
        h.max_tiles = L.max_tiles;
        // few workgroups: each adds its bins to the global histogram once
        const int64_t hist_blocks = std::min<int64_t>(std::max<int64_t>((n + 4095) / 4096, 1), 256);
        timing_begin(hist_id, stream);
        hipLaunchKernelGGL(k_sort_hist<K>, dim3(uint32_t(hist_blocks)), dim3(kHistThreads), 0, stream, h);
        timing_end(hist_id, stream);
    }
    for (int p = 0; p < L.passes; ++p) {
        const K* pk = p == 0 ? kin : ((L.passes - p) % 2 == 0 ? kout : alt_keys);
        const uint32_t* pv = p == 0 ? vin : ((L.passes - p) % 2 == 0 ? vout : L.alt_vals);
        const bool to_out = (L.passes - 1 - p) % 2 == 0;
        K* ok = to_out ? kout : alt_keys;
        uint32_t* ov = to_out ? vout : L.alt_vals;
        const int shift = begin_bit + p * L.r;
        const int bits = std::min(L.r, end_bit - shift);
        PassLaunch<K> c;
        c.L = &L;
        c.d_status = d_status;
        c.stream = stream;
        c.ua = UpArgs<K>{pk, n, d_n, d_status, shift, L.table, L.max_tiles, nullptr, 0};
        if (L.wait_free) {
            c.ua.clear = static_cast<uint32_t*>(L.table_scan);
            c.ua.clear_words = scan_sync_words(int64_t(1 << bits) * L.max_tiles, kTableItems);
        }
        c.da = DownArgs<K>{pk, pv, ok, ov, n, d_n, d_status, shift, L.table, L.max_tiles};
        c.pa.kin = pk;
        c.pa.vin = pv;
        c.pa.kout = ok;
        c.pa.vout = ov;
        c.pa.cap = n;
        c.pa.d_n = d_n;
        c.pa.d_status_rw = const_cast<int32_t*>(d_status);
        c.pa.d_status = d_status;
        c.pa.shift = shift;
        c.pa.hist = L.wait_free ? nullptr : L.hist + p * L.radix;
        c.pa.status = L.wait_free ? nullptr : L.status + int64_t(p) * L.max_tiles * L.radix;
        timing_begin(pass_id, stream);
        if (L.items == kItemsSmall) run_pass_bits<kItemsSmall, K>(c, bits);
        else if (L.items == kItemsMid) run_pass_bits<kItemsMid, K>(c, bits);
        else run_pass_bits<kItemsLarge, K>(c, bits);
        timing_end(pass_id, stream);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sort(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout, int64_t n,
                       const int64_t* d_n, const int32_t* d_status, int32_t begin_bit, int32_t end_bit,
                       int32_t radix_bits, void* ws, hipStream_t stream, bool timed, bool sparse, bool precleared,
                       bool hist_ready) {
    return launch_sort_t<uint64_t>(kin, vin, kout, vout, n, d_n, d_status, begin_bit, end_bit, radix_bits, ws, stream,
                                   timed, sparse, precleared, hist_ready);
}

hipError_t launch_sort(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, int64_t n,
                       const int64_t* d_n, const int32_t* d_status, int32_t begin_bit, int32_t end_bit,
                       int32_t radix_bits, void* ws, hipStream_t stream, bool timed, bool sparse, bool precleared,
                       bool hist_ready) {
    return launch_sort_t<uint32_t>(kin, vin, kout, vout, n, d_n, d_status, begin_bit, end_bit, radix_bits, ws, stream,
                                   timed, sparse, precleared, hist_ready);
}

}  // namespace ws
