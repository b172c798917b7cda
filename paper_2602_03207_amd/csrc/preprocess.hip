// Pre-processing stage (Sec. 3.2) and key emission.
//
// k_preprocess  one thread per (view, Gaussian): opacity cull, projection,
//               bounding-box cull, SH colour; writes the 48-byte splat record
//               of visible splats and tiles_touched of every splat.
// compaction    list of the visible (view, Gaussian) entries in index order,
//               the survivors "written into a buffer" of Sec. 3.2 (prefix sum
//               of the visibility flags).  With WS_FLAG_DEPTH_FIRST each
//               entry's fp32 depth bits are written too and the list is then
//               stably sorted by depth.
// counts        prefix sum of the listed entries' tile counts: each entry's
//               first pair, the total M, and for every emission block of the
//               output the entry that owns its first pair.
// k_emit        one workgroup per block of 512, 1024 or 2048 pairs (by the
//               pair capacity), in rounds of up to 256 entries:
//               loads the entries that cover the round's pairs, finds each
//               pair's owner by marking the entry starts in LDS and taking a
//               running maximum, and writes key = (tile << 32) | depth bits
//               (the tile alone as a 32-bit key with WS_FLAG_KEYS32, where the
//               depth order is the emission order), value = Gaussian id with
//               coalesced stores.  With bins of tiles as key cells the bits
//               above the bin id carry, where they fit, the mask of the bin's
//               tiles that the splat's rectangle meets (bit row * bin_x + col).  Work per
//               workgroup is fixed, whatever the size of the splats.
// Both prefix sums are those of scan.h (one pass with look-back up to 1024
// workgroups, else the wait-free three-level scan).  k_preprocess zeroes the
// look-back words of both scans and of the depth sort on its way, so none of
// them needs a clearing launch.
#include "project.h"
#include "scan.h"
#include "ws_internal.h"

namespace ws {
namespace {

constexpr int kPreThreads = 256;
constexpr int kEmitThreads = 256;
constexpr int kEmitSlots = kEmitThreads;  // entries loaded per round
// Pairs per emission workgroup: kEmitThreads x (2, 4 or 8) by the pair
// capacity.  Small frames (a 1080p view's 1.1 M bin pairs) spread over more
// workgroups; large ones (49 M pairs at 4K) keep 2 048-pair blocks, where
// smaller blocks cost more in per-block overhead than they gain.
inline int emit_items_for(int64_t capacity) {
    return capacity <= (int64_t(1) << 21) ? 2 : (capacity <= (int64_t(1) << 23) ? 4 : 8);
}
// Items per thread of the two prefix sums: the visibility flags of every
// entry (large blocks, a short look-back) and the tile counts of the listed
// entries (smaller blocks: few entries are listed and each count takes two
// dependent loads).
constexpr int kCompactItems = 16;
constexpr int kCountItems = 4;
// The depth sort of depth-first emission: 31 key bits in 4 passes of 8 bits.
constexpr int kDepthPasses = 4, kDepthRadixBits = 8, kDepthRadix = 1 << kDepthRadixBits;

struct PreprocessWs {
    uint32_t* list_a;       // [V n] visible entries in index order
    uint32_t* list_b;       // [V n] the same, sorted by depth (depth-first mode)
    uint32_t* depth;        // [V n] fp32 depth bits of every visible entry (depth-first mode)
    uint32_t* dkey_a;       // [V n] fp32 depth bits of list_a (depth-first mode)
    uint32_t* dkey_b;
    uint32_t* offsets;      // [V n] first pair of each list entry
    uint32_t* first_entry;  // [emit blocks] list entry owning each block's first pair
    void* scan_a;           // workspaces of the two prefix sums
    void* scan_b;
    int64_t* d_nvis;
    void* sort_ws;
    int64_t total, emit_blocks;
    int32_t emit_items;  // pairs per emission workgroup / kEmitThreads
};

size_t layout(void* ws, int64_t n, int32_t n_views, int64_t capacity, bool depth_first, PreprocessWs* out) {
    PreprocessWs p{};
    p.total = n * n_views;
    const int64_t ents = std::max<int64_t>(p.total, 1);
    p.emit_items = emit_items_for(capacity);
    const int64_t emit_pairs = int64_t(kEmitThreads) * p.emit_items;
    p.emit_blocks = std::max<int64_t>((capacity + emit_pairs - 1) / emit_pairs, 1);
    char* base = static_cast<char*>(ws);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* ptr = base ? base + off : nullptr;
        off += align_up(bytes);
        return ptr;
    };
    p.d_nvis = reinterpret_cast<int64_t*>(take(16));
    p.scan_a = take(scan_workspace(ents, kCompactItems));
    p.scan_b = take(scan_workspace(ents, kCountItems));
    p.list_a = reinterpret_cast<uint32_t*>(take(size_t(ents) * 4));
    p.offsets = reinterpret_cast<uint32_t*>(take(size_t(ents) * 4));
    p.first_entry = reinterpret_cast<uint32_t*>(take(size_t(p.emit_blocks) * 4));
    if (depth_first) {
        p.list_b = reinterpret_cast<uint32_t*>(take(size_t(ents) * 4));
        p.depth = reinterpret_cast<uint32_t*>(take(size_t(ents) * 4));
        p.dkey_a = reinterpret_cast<uint32_t*>(take(size_t(ents) * 4));
        p.dkey_b = reinterpret_cast<uint32_t*>(take(size_t(ents) * 4));
        p.sort_ws = take(sort_workspace(ents, 0, 31, kDepthRadixBits, true, 4));
    }
    if (out) *out = p;
    return off;
}

// Workgroup order: the grid holds gx8 blocks of Gaussians (gx rounded up to a
// multiple of 8) for each of the V views.  Workgroups are dealt to the 8 XCDs
// in turn, so workgroup p runs on XCD p % 8; its (block, view) is chosen so
// that each XCD takes the V views of one block one after the other (block
// p % 8 + 8 (j / V), view j % V, j = p / 8): a block's parameters are then
// read from memory once and served to its other views by that XCD's L2.
template <int DEG>
__global__ __launch_bounds__(kPreThreads) void k_preprocess(GaussPtrs g, const ws_camera* __restrict__ cams, KOpts o,
                                                           int32_t n_views, ws_splat* __restrict__ splats,
                                                           uint32_t* __restrict__ tiles_touched,
                                                           uint32_t* __restrict__ depth, ClearList clr) {
    const uint32_t j = blockIdx.x >> 3;
    const int32_t v = int32_t(j % uint32_t(n_views));
    const int64_t blk = int64_t(blockIdx.x & 7u) + 8 * int64_t(j / uint32_t(n_views));
    const int64_t i = blk * kPreThreads + threadIdx.x;
    // the look-back words of the scans and of the depth sort that follow, and the status word
    clear_words(clr, int64_t(blockIdx.x) * kPreThreads + threadIdx.x, int64_t(gridDim.x) * kPreThreads);
    if (i >= g.n) return;
    const ws_camera& cam = cams[v];
    ProjState st;
    const bool vis = compute_projection<DEG>(g, i, cam, o, st);
    const int64_t vi = int64_t(v) * g.n + i;
    tiles_touched[vi] = vis ? st.tiles : 0u;
    if (!vis) return;
    const uint32_t r01 = uint32_t(st.rect[0]) | (uint32_t(st.rect[1]) << 16);
    const uint32_t r23 = uint32_t(st.rect[2]) | (uint32_t(st.rect[3]) << 16);
    if (o.flags & WS_FLAG_PACKED) {  // 32-byte ws_splat_packed records
        float ax[4];
        ellipse_axes(st.a, st.b, st.c, st.det, ax);
        const uint32_t a01 = half_bits(ax[0]) | (half_bits(ax[1]) << 16);
        const uint32_t a23 = half_bits(ax[2]) | (half_bits(ax[3]) << 16);
        const uint32_t rgba = unorm8(fminf(st.rgb[0], 1.f)) | (unorm8(fminf(st.rgb[1], 1.f)) << 8) |
                              (unorm8(fminf(st.rgb[2], 1.f)) << 16) | (unorm8(st.sigma) << 24);
        float4* rec = reinterpret_cast<float4*>(splats) + 2 * vi;
        rec[0] = make_float4(st.u, st.v, __uint_as_float(a01), __uint_as_float(a23));
        rec[1] = make_float4(__uint_as_float(rgba), st.z32, __uint_as_float(r01), __uint_as_float(r23));
    } else {
        float4* rec = reinterpret_cast<float4*>(splats + vi);
        rec[0] = make_float4(st.u, st.v, st.A, st.B);
        rec[1] = make_float4(st.C, st.sigma, st.rgb[0], st.rgb[1]);
        rec[2] = make_float4(st.rgb[2], st.z32, __uint_as_float(r01), __uint_as_float(r23));
    }
    // a dense copy of the depth, so that the compaction reads it coalesced
    // rather than one word out of every 48-byte record
    if (depth) depth[vi] = __float_as_uint(st.z32);
}

// ---- compaction: prefix sum of the visibility flags
struct FlagItem {
    uint32_t tiles, depth;  // depth bits are read only for visible entries (depth-first mode)
};
struct FlagLoad {
    using Item = FlagItem;
    const uint32_t* tiles_touched;
    const uint32_t* depth;  // null unless depth-first
    __device__ FlagItem operator()(int64_t i) const { return FlagItem{tiles_touched[i], depth ? depth[i] : 0u}; }
    __device__ static uint64_t value(const FlagItem& it) { return it.tiles != 0u ? 1u : 0u; }
};
struct CompactStore {
    uint32_t* list;
    uint32_t* dkeys;  // null unless depth-first
    __device__ void operator()(int64_t i, uint64_t pos, const FlagItem& it) const {
        if (it.tiles == 0u) return;
        list[pos] = uint32_t(i);
        if (dkeys) dkeys[pos] = it.depth;
    }
};

// ---- depth-first compaction: one kernel lists the visible entries with their
// depth keys and prepares the depth sort that follows.  Block b takes `rounds`
// consecutive chunks of 4096 entries (16 per thread, wave-striped; enough
// rounds that at most kCompactMaxBlocks blocks cover the input), counts their
// visible entries and finds its offset by the decoupled look-back of scan.h
// (block b waits only for lower blocks, which each XCD starts first; bounded
// wait; the look-back's latency grows with the block count, hence the cap),
// then writes the list entries and depth keys (with several rounds the
// entries are read again, from the cache, for the writes).  On the way it
// counts the depth digits of its visible entries for every pass of the depth
// sort (LDS, then one global add per non-zero bin) and zeroes the sort's
// look-back words of the sort tiles its entries land in, so the sort needs no
// histogram launch.
constexpr int kCompactThreads = 256;
constexpr int kCompactBlock = kCompactThreads * kCompactItems;
constexpr int kCompactWaves = kCompactThreads / kWave;
constexpr int64_t kCompactMaxBlocks = 1024;
constexpr int kCompactMaxRounds = 64;

struct CompactArgs {
    const uint32_t* tiles_touched;
    const uint32_t* depth;
    uint32_t* list;
    uint32_t* dkeys;
    int64_t total;
    int32_t rounds;  // chunks of kCompactBlock entries per block
    uint64_t* look;  // [blocks] look-back words, zeroed by k_preprocess
    int64_t* d_nvis;
    int32_t* d_status;
    SortHistWords sw;  // the depth sort's histograms (zeroed by k_preprocess) and look-back words
};

inline int32_t compact_rounds(int64_t total) {
    const int64_t chunks = (std::max<int64_t>(total, 1) + kCompactBlock - 1) / kCompactBlock;
    return int32_t(std::min<int64_t>((chunks + kCompactMaxBlocks - 1) / kCompactMaxBlocks, kCompactMaxRounds));
}
inline int64_t compact_blocks_of(int64_t total) {
    const int64_t per = int64_t(kCompactBlock) * compact_rounds(total);
    return (std::max<int64_t>(total, 1) + per - 1) / per;
}

// Loads one chunk's visibility flags and depth keys (16 per thread).
__device__ __forceinline__ void compact_load(const CompactArgs& a, int64_t wbase, uint32_t* tt, uint32_t* dk) {
#pragma unroll
    for (int j = 0; j < kCompactItems; ++j) {
        const int64_t i = wbase + j * kWave;
        const int64_t ic = i < a.total ? i : a.total - 1;
        tt[j] = a.tiles_touched[ic];
        dk[j] = a.depth[ic];
    }
#pragma unroll
    for (int j = 0; j < kCompactItems; ++j) tt[j] = (wbase + j * kWave < a.total && tt[j] != 0u) ? 1u : 0u;
}

template <bool MULTI>
__global__ __launch_bounds__(kCompactThreads) void k_compact(CompactArgs a) {
    constexpr int kPerWave = kCompactItems * kWave;
    constexpr int bins = kDepthPasses * kDepthRadix;
    __shared__ uint32_t s_hist[bins];
    __shared__ uint32_t s_cnt[kCompactMaxRounds * kCompactWaves];  // visible entries per (round, wave)
    __shared__ uint64_t s_excl;
    if (*a.d_status != 0) return;
    const int64_t per_block = int64_t(kCompactBlock) * a.rounds;
    const int64_t nb = (a.total + per_block - 1) / per_block;
    if (int64_t(blockIdx.x) >= nb) return;
    const int64_t b = blockIdx.x;
    for (int k = threadIdx.x; k < bins; k += kCompactThreads) s_hist[k] = 0;
    const int wave = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    __syncthreads();  // the histogram's zeroing before the adds
    uint32_t tt[kCompactItems], dk[kCompactItems];
    const int rounds = MULTI ? a.rounds : 1;
    for (int r = 0; r < rounds; ++r) {
        const int64_t wbase = b * per_block + int64_t(r) * kCompactBlock + int64_t(wave) * kPerWave + lane;
        compact_load(a, wbase, tt, dk);
        uint32_t cnt = 0;
#pragma unroll
        for (int j = 0; j < kCompactItems; ++j) {
            cnt += uint32_t(__popcll(__ballot(tt[j] != 0u)));
            // depth digits of every pass (bit 31 of a positive depth is 0)
            if (tt[j]) {
#pragma unroll
                for (int p = 0; p < kDepthPasses; ++p)
                    atomicAdd(&s_hist[p * kDepthRadix + ((dk[j] >> (p * kDepthRadixBits)) & (kDepthRadix - 1))], 1u);
            }
        }
        if (lane == 0) s_cnt[r * kCompactWaves + wave] = cnt;
    }
    __syncthreads();
    uint64_t block_sum = 0;
    for (int k = 0; k < rounds * kCompactWaves; ++k) block_sum += s_cnt[k];
    if (wave == 0) {
        if (lane == 0) store_agent(&a.look[b], (b == 0 ? kScanInc : kScanAgg) | block_sum);
        uint64_t excl = 0;
        if (b > 0) {
            int64_t k = b - 1;  // lane l reads predecessor k - l
            uint32_t spins = 0;
            while (true) {
                const int64_t kk = k - int64_t(lane);
                uint64_t st = kk >= 0 ? load_agent(&a.look[kk]) : kScanInc;
                uint64_t need = 0, incm = 0;
                while (true) {
                    incm = __ballot((st >> 62) == 2);
                    const uint64_t zero = __ballot((st >> 62) == 0);
                    need = incm ? ((incm & (~incm + 1)) << 1) - 1 : ~uint64_t(0);
                    if ((zero & need) == 0) break;
                    if (++spins > kSpinLimit) {
                        if (lane == 0) atomicExch(a.d_status, int32_t(WS_ERR_SPIN_LIMIT));
                        need = 0;
                        incm = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    if ((st >> 62) == 0) st = load_agent(&a.look[kk]);
                }
                const uint64_t part = ((need >> lane) & 1) ? (st & kScanVal) : 0;
                excl += wave_sum(part);
                if (incm) break;
                k -= kWave;
            }
            if (lane == 0) store_agent(&a.look[b], kScanInc | (excl + block_sum));
        }
        if (lane == 0) {
            s_excl = excl;
            if (b == nb - 1) *a.d_nvis = int64_t(excl + block_sum);
        }
    }
    __syncthreads();
    uint64_t off = s_excl;
    for (int r = 0; r < rounds; ++r) {
        uint64_t woff = 0, rsum = 0;
        for (int w = 0; w < kCompactWaves; ++w) {
            const uint32_t c = s_cnt[r * kCompactWaves + w];
            woff += w < wave ? c : 0u;
            rsum += c;
        }
        const int64_t wbase = b * per_block + int64_t(r) * kCompactBlock + int64_t(wave) * kPerWave + lane;
        if (MULTI) compact_load(a, wbase, tt, dk);  // again, from the cache
        uint64_t pos = off + woff;
#pragma unroll
        for (int j = 0; j < kCompactItems; ++j) {
            const uint64_t m = __ballot(tt[j] != 0u);
            if (tt[j]) {
                const uint64_t q = pos + lanes_below(m);
                a.list[q] = uint32_t(wbase + j * kWave);
                a.dkeys[q] = dk[j];
            }
            pos += uint64_t(__popcll(m));
        }
        off += rsum;
    }
    for (int k = threadIdx.x; k < bins; k += kCompactThreads)
        if (s_hist[k]) atomicAdd(&a.sw.hist[k], s_hist[k]);
    // the depth sort's look-back words of the sort tiles this block's entries land in
    if (block_sum > 0) {
        const int64_t t0 = int64_t(s_excl) / a.sw.tile, t1 = int64_t(s_excl + block_sum - 1) / a.sw.tile;
        const uint32_t words = uint32_t(t1 - t0 + 1) * kDepthRadix;  // per pass, a few tiles
#pragma unroll
        for (int p = 0; p < kDepthPasses; ++p) {
            uint32_t* st = a.sw.status + (int64_t(p) * a.sw.max_tiles + t0) * kDepthRadix;
            for (uint32_t w = threadIdx.x; w < words; w += kCompactThreads) st[w] = 0u;
        }
    }
}

// ---- counts: prefix sum of the listed entries' tile counts
struct CountLoad {
    using Item = uint64_t;
    const uint32_t* tiles_touched;
    const uint32_t* list;
    __device__ uint64_t operator()(int64_t e) const { return tiles_touched[list[e]]; }
    __device__ static uint64_t value(uint64_t c) { return c; }
};
struct CountStore {
    uint32_t* offsets;
    uint32_t* first_entry;
    int64_t emit_blocks;
    uint32_t emit_pairs;  // pairs per emission block
    __device__ void operator()(int64_t e, uint64_t s, uint64_t cnt) const {
        offsets[e] = uint32_t(s);
        if (cnt == 0) return;
        // every output block whose first pair falls inside [s, s + cnt) starts in entry e
        const uint64_t b_lo = (s + emit_pairs - 1) / emit_pairs;
        const uint64_t b_hi = (s + cnt - 1) / emit_pairs;
        for (uint64_t b = b_lo; b <= b_hi && int64_t(b) < emit_blocks; ++b) first_entry[b] = uint32_t(e);
    }
};

struct EmitArgs {
    const float4* splats;  // records of rec_f4 float4s; float4 rec_tail of each holds (., depth, rect01, rect23)
    int32_t rec_f4, rec_tail;
    const ws_camera* cams;
    int32_t n_views;
    const uint32_t* list;
    const uint32_t* offsets;
    const uint32_t* first_entry;
    const int64_t* d_nvis;
    const int64_t* d_num_pairs;
    int32_t* d_status;
    int64_t n;
    int64_t capacity;
    int32_t tile_w, tile_h;        // pixel size of a key cell (tile or bin)
    uint32_t tw_shift, th_shift;  // log2 of the cell size
    uint32_t tws, ths;            // log2 of the tile size (bins only)
    uint32_t bxs, bys;            // log2 of the bin size in tiles (bins only)
    int32_t mask_shift;           // bit of the cell word where the coverage mask starts, -1: no mask
    void* keys;                   // uint64_t, or uint32_t cell ids (K32)
    uint32_t* values;
};

// The tiles of bin (cx, cy) that a splat's pixel rectangle (x0 | x1 << 16,
// y0 | y1 << 16) meets, as bits row * bin_x + col of the bin's tiles.  The bin
// is one the rectangle meets, so the column and row spans are not empty; the
// rectangle is clipped to the image, so no bit names a tile past its edge.
__device__ __forceinline__ uint32_t bin_coverage(uint32_t prx, uint32_t pry, uint32_t cx, uint32_t cy,
                                                 const EmitArgs& a) {
    const uint32_t t0x = (prx & 0xffffu) >> a.tws, t1x = (prx >> 16) >> a.tws;
    const uint32_t t0y = (pry & 0xffffu) >> a.ths, t1y = (pry >> 16) >> a.ths;
    const uint32_t bx0 = cx << a.bxs, by0 = cy << a.bys;  // the bin's first tile
    const uint32_t bx1 = bx0 + (1u << a.bxs) - 1u, by1 = by0 + (1u << a.bys) - 1u;
    if (t1x < bx0 || t0x > bx1 || t1y < by0 || t0y > by1) return 0u;  // (not reached)
    const uint32_t c0 = max(t0x, bx0) - bx0, c1 = min(t1x, bx1) - bx0;  // <= 7
    const uint32_t r0 = max(t0y, by0) - by0, r1 = min(t1y, by1) - by0;  // <= 7
    const uint32_t row = (0xffffffffu >> (31u - c1)) & (0xffffffffu << c0);  // bits c0..c1
    uint32_t m = 0;
    for (uint32_t r = r0; r <= r1; ++r) m |= row << (r << a.bxs);
    return m;
}

// Inclusive prefix maximum over the 64 lanes of a wave (values >= 0), by the
// DPP steps of wave_inclusive_scan.
__device__ __forceinline__ uint32_t wave_inclusive_max(uint32_t v) {
    v = max(v, dpp_move<0x111>(v));        // row_shr 1
    v = max(v, dpp_move<0x112>(v));        // row_shr 2
    v = max(v, dpp_move<0x114>(v));        // row_shr 4
    v = max(v, dpp_move<0x118>(v));        // row_shr 8: prefix maxima within each row
    v = max(v, dpp_move<0x142, 0xa>(v));   // row_bcast 15 into rows 1 and 3
    v = max(v, dpp_move<0x143, 0xc>(v));   // row_bcast 31 into rows 2 and 3
    return v;
}

template <bool K32, bool MASK, int EI>
__global__ __launch_bounds__(kEmitThreads) void k_emit(EmitArgs a) {
    constexpr int kEmitItems = EI, kEmitPairs = kEmitThreads * EI;
    __shared__ uint32_t s_owner[kEmitPairs];
    __shared__ uint32_t s_start[kEmitSlots];
    __shared__ uint32_t s_gid[kEmitSlots];
    __shared__ uint32_t s_depth[kEmitSlots];
    __shared__ uint32_t s_trx[kEmitSlots];
    __shared__ uint32_t s_try[kEmitSlots];
    __shared__ uint32_t s_tbase[kEmitSlots];
    __shared__ uint32_t s_tilesx[kEmitSlots];
    __shared__ uint32_t s_magic[kEmitSlots];  // floor((2^32 - 1) / tile-rectangle width)
    __shared__ uint32_t s_prx[MASK ? kEmitSlots : 1], s_pry[MASK ? kEmitSlots : 1];  // pixel rectangle
    __shared__ uint32_t s_scan[kEmitThreads / kWave + 1];
    __shared__ int64_t s_hi;
    __shared__ uint32_t s_vtoff[kEmitThreads], s_vtx[kEmitThreads];
    if (*a.d_status != 0) return;
    const int64_t m = *a.d_num_pairs;
    if (m > a.capacity) {  // the caller's buffers are too small: report, write nothing
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(a.d_status, int32_t(WS_ERR_CAPACITY));
        return;
    }
    const int64_t p0 = int64_t(blockIdx.x) * kEmitPairs;
    if (p0 >= m) return;
    const int64_t p1 = min(p0 + kEmitPairs, m);
    const int64_t nvis = *a.d_nvis;  // >= 1: there are pairs
    int64_t e = a.first_entry[blockIdx.x];
    // first tile id and tiles per row of every view: one view needs no table;
    // up to one view per thread they come from a table in LDS; more views fall
    // back to summing the cameras per entry
    const bool one_view = a.n_views == 1;
    const uint32_t tx_one = uint32_t(ceil_div(a.cams[0].width, a.tile_w));
    const bool view_table = !one_view && a.n_views <= kEmitThreads;
    if (view_table) {
        uint32_t tiles = 0, tx = 0;
        if (int32_t(threadIdx.x) < a.n_views) {
            tx = uint32_t(ceil_div(a.cams[threadIdx.x].width, a.tile_w));
            tiles = tx * uint32_t(ceil_div(a.cams[threadIdx.x].height, a.tile_h));
        }
        uint32_t total;
        const uint32_t toff = block_exclusive_scan<kEmitThreads>(tiles, s_scan, &total);
        s_vtoff[threadIdx.x] = toff;
        s_vtx[threadIdx.x] = tx;
    }
    // Rounds: entries e, e + 1, ..., e + kEmitSlots - 1 (entry e owns pair lo)
    // cover the pairs [lo, hi), hi = the first pair of entry e + kEmitSlots
    // (or p1).  Entry starts strictly increase: every listed entry has pairs.
    int64_t lo = p0;
    while (lo < p1) {
        for (int q = threadIdx.x; q < kEmitPairs; q += kEmitThreads) s_owner[q] = 0;
        const int slot = threadIdx.x;
        const int64_t ent = e + slot;
        // the entry's start and list index, and the round's end, loaded together
        const int64_t ec = ent < nvis ? ent : nvis - 1;
        const uint32_t start = a.offsets[ec];
        const uint32_t idx = a.list[ec];
        const int64_t next = e + kEmitSlots;
        const uint32_t next_start = a.offsets[next < nvis ? next : nvis - 1];
        __syncthreads();
        const bool in = ent < nvis && int64_t(start) < p1;
        if (in) {
            const int64_t view = int64_t(idx / uint32_t(a.n));  // V n < 2^32
            const float4 r2 = a.splats[int64_t(idx) * a.rec_f4 + a.rec_tail];
            const uint32_t r01 = __float_as_uint(r2.z), r23 = __float_as_uint(r2.w);
            uint32_t tbase, tilesx;
            if (one_view) {
                tbase = 0;
                tilesx = tx_one;
            } else if (view_table) {
                tbase = s_vtoff[view];
                tilesx = s_vtx[view];
            } else {
                int64_t toff, ioff;
                view_offsets(a.cams, int32_t(view), a.tile_w, a.tile_h, &toff, &ioff);
                tbase = uint32_t(toff);
                tilesx = uint32_t(ceil_div(a.cams[view].width, a.tile_w));
            }
            s_start[slot] = start;
            s_gid[slot] = uint32_t(int64_t(idx) - view * a.n);
            s_depth[slot] = __float_as_uint(r2.y);
            // cell sizes are powers of two
            const uint32_t tx0 = (r01 & 0xffffu) >> a.tw_shift, tx1 = (r01 >> 16) >> a.tw_shift;
            s_trx[slot] = tx0 | (tx1 << 16);
            s_try[slot] = ((r23 & 0xffffu) >> a.th_shift) | (((r23 >> 16) >> a.th_shift) << 16);
            s_tbase[slot] = tbase;
            s_tilesx[slot] = tilesx;
            s_magic[slot] = 0xffffffffu / (tx1 - tx0 + 1);
            if (MASK) {
                s_prx[slot] = r01;
                s_pry[slot] = r23;
            }
            if (slot > 0) s_owner[int64_t(start) - p0] = uint32_t(slot);
        }
        if (threadIdx.x == 0) s_hi = next < nvis ? min(p1, int64_t(next_start)) : p1;
        __syncthreads();
        const int64_t hi = s_hi;
        // owner of pair q = the largest slot that starts at or before q (slot 0
        // owns lo; marks before lo were cleared)
        uint32_t own[kEmitItems];
        uint32_t run = 0;
#pragma unroll
        for (int j = 0; j < kEmitItems; ++j) {
            run = max(run, s_owner[threadIdx.x * kEmitItems + j]);
            own[j] = run;
        }
        // exclusive max-scan of the threads' last owners: inside the wave by DPP
        // (prefix maxima within rows of 16 by shifts, then the row broadcasts),
        // across the waves through LDS
        {
            const uint32_t v = wave_inclusive_max(run);
            const uint32_t lane = lane_id();
            const int wave = threadIdx.x / kWave;
            if (lane == kWave - 1) s_scan[wave] = v;
            __syncthreads();
            uint32_t before = dpp_move<0x138>(v);  // wave_shr 1: the previous lane's prefix, 0 in lane 0
            for (int w = 0; w < wave; ++w) before = max(before, s_scan[w]);
#pragma unroll
            for (int j = 0; j < kEmitItems; ++j) own[j] = max(own[j], before);
        }
        // hand the owners over through LDS so that consecutive lanes write
        // consecutive pairs (the scan above runs on consecutive pairs per thread)
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kEmitItems; ++j) s_owner[threadIdx.x * kEmitItems + j] = own[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kEmitItems; ++j) {
            const int q = j * kEmitThreads + threadIdx.x;
            const int64_t p = p0 + q;
            if (p >= lo && p < hi) {
                const uint32_t s = s_owner[q];
                const uint32_t k = uint32_t(p - int64_t(s_start[s]));
                const uint32_t xr = s_trx[s], yr = s_try[s];
                const uint32_t tx0 = xr & 0xffffu, tx1 = xr >> 16, ty0 = yr & 0xffffu;
                const uint32_t w = tx1 - tx0 + 1;
                // k / w by a multiply-high with floor((2^32 - 1) / w), which
                // undershoots by at most 2 for any 32-bit k; then corrected
                uint32_t row = __umulhi(k, s_magic[s]), col = k - row * w;
                if (col >= w) {
                    ++row;
                    col -= w;
                }
                if (col >= w) {
                    ++row;
                    col -= w;
                }
                const uint64_t tile = uint64_t(s_tbase[s]) + uint64_t(ty0 + row) * s_tilesx[s] + (tx0 + col);
                uint32_t word = uint32_t(tile);  // the cell id (< 2^32; below 2^mask_shift with a mask)
                if (MASK) word |= bin_coverage(s_prx[s], s_pry[s], tx0 + col, ty0 + row, a) << a.mask_shift;
                if (K32) static_cast<uint32_t*>(a.keys)[p] = word;
                else static_cast<uint64_t*>(a.keys)[p] = (uint64_t(word) << 32) | s_depth[s];
                a.values[p] = s_gid[s];
            }
        }
        e += kEmitSlots;
        lo = hi;
        __syncthreads();  // the next round reuses the LDS
    }
}

template <int EI>
void launch_emit(const EmitArgs& ea, bool k32, bool mask, int64_t blocks, hipStream_t stream) {
    const dim3 eg(static_cast<uint32_t>(blocks)), eb(kEmitThreads);
    if (k32 && mask) hipLaunchKernelGGL((k_emit<true, true, EI>), eg, eb, 0, stream, ea);
    else if (k32) hipLaunchKernelGGL((k_emit<true, false, EI>), eg, eb, 0, stream, ea);
    else if (mask) hipLaunchKernelGGL((k_emit<false, true, EI>), eg, eb, 0, stream, ea);
    else hipLaunchKernelGGL((k_emit<false, false, EI>), eg, eb, 0, stream, ea);
}

}  // namespace

size_t preprocess_workspace(int64_t n, int32_t n_views, int64_t capacity, uint32_t flags) {
    return layout(nullptr, n, n_views, capacity, (flags & WS_FLAG_DEPTH_FIRST) != 0, nullptr);
}

hipError_t launch_preprocess(const GaussPtrs& g, const ws_camera* d_cams, int32_t n_views, const KOpts& o,
                             ws_splat* splats, uint32_t* tiles_touched, void* keys, uint32_t* values,
                             int64_t capacity, int64_t* d_num_pairs, int32_t* d_status, void* ws,
                             hipStream_t stream) {
    const bool depth_first = (o.flags & WS_FLAG_DEPTH_FIRST) != 0;
    PreprocessWs pw;
    layout(ws, g.n, n_views, capacity, depth_first, &pw);
    const uint32_t gx = uint32_t(std::max<int64_t>((g.n + kPreThreads - 1) / kPreThreads, 1));
    const int64_t ents = std::max<int64_t>(pw.total, 1);
    ClearList clr;
    // depth-first: k_compact's look-back words (one 64-bit word per block); otherwise those of the scan
    const int64_t compact_blocks = compact_blocks_of(ents);
    clr.add(pw.scan_a, depth_first ? 2 * compact_blocks : scan_sync_words(pw.total, kCompactItems));
    if (depth_first) sort_sync_words(pw.sort_ws, ents, 0, 31, kDepthRadixBits, true, 4, &clr);
    clr.add(pw.scan_b, scan_sync_words(ents, kCountItems, true));
    // a frame starts with a clean status word (no kernel of this launch reads it)
    clr.add(d_status, 1);
    timing_begin(WS_KERNEL_PREPROCESS, stream);
    const dim3 pgrid(uint32_t((gx + 7) / 8 * 8) * uint32_t(n_views));
    switch (o.sh_degree) {
        case 0: hipLaunchKernelGGL(k_preprocess<0>, pgrid, dim3(kPreThreads), 0, stream, g, d_cams, o, n_views,
                                   splats, tiles_touched, pw.depth, clr); break;
        case 1: hipLaunchKernelGGL(k_preprocess<1>, pgrid, dim3(kPreThreads), 0, stream, g, d_cams, o, n_views,
                                   splats, tiles_touched, pw.depth, clr); break;
        case 2: hipLaunchKernelGGL(k_preprocess<2>, pgrid, dim3(kPreThreads), 0, stream, g, d_cams, o, n_views,
                                   splats, tiles_touched, pw.depth, clr); break;
        default: hipLaunchKernelGGL(k_preprocess<3>, pgrid, dim3(kPreThreads), 0, stream, g, d_cams, o, n_views,
                                    splats, tiles_touched, pw.depth, clr); break;
    }
    timing_end(WS_KERNEL_PREPROCESS, stream);

    timing_begin(WS_KERNEL_SCAN_EMIT, stream);
    const uint32_t* list = pw.list_a;
    if (depth_first) {
        // compaction of the visible entries with their depth keys (count to d_nvis), which also
        // prepares the depth sort: its digit histograms and look-back words
        CompactArgs ca;
        ca.tiles_touched = tiles_touched;
        ca.depth = pw.depth;
        ca.list = pw.list_a;
        ca.dkeys = pw.dkey_a;
        ca.total = ents;
        ca.rounds = compact_rounds(ents);
        ca.look = static_cast<uint64_t*>(pw.scan_a);
        ca.d_nvis = pw.d_nvis;
        ca.d_status = d_status;
        ca.sw = sort_hist_words(pw.sort_ws, ents, 0, 31, kDepthRadixBits, true, 4);
        if (ca.sw.passes != kDepthPasses || ca.sw.radix != kDepthRadix) std::abort();  // a programming error
        if (ca.rounds > 1)
            hipLaunchKernelGGL(k_compact<true>, dim3(uint32_t(compact_blocks)), dim3(kCompactThreads), 0, stream, ca);
        else
            hipLaunchKernelGGL(k_compact<false>, dim3(uint32_t(compact_blocks)), dim3(kCompactThreads), 0, stream, ca);
        // stable sort of the visible entries by depth: positive fp32 bits order like the values
        // the visible entries are typically a small fraction of all (view, Gaussian) entries
        const hipError_t e = launch_sort(pw.dkey_a, pw.list_a, pw.dkey_b, pw.list_b, ents, pw.d_nvis, d_status, 0, 31,
                                         kDepthRadixBits, pw.sort_ws, stream, false, true, true, true);
        if (e != hipSuccess) return e;
        list = pw.list_b;
    } else {
        // compaction of the visible entries (count to d_nvis)
        launch_scan<uint64_t, kCompactItems>(FlagLoad{tiles_touched, nullptr}, CompactStore{pw.list_a, nullptr},
                                             pw.total, nullptr, d_status, pw.scan_a,
                                             reinterpret_cast<uint64_t*>(pw.d_nvis), stream, true);
    }
    // pair offsets of the listed entries (total to d_num_pairs)
    launch_scan<uint64_t, kCountItems>(CountLoad{tiles_touched, list}, CountStore{pw.offsets, pw.first_entry, pw.emit_blocks,
                                                                       uint32_t(kEmitThreads * pw.emit_items)},
                          ents, pw.d_nvis, d_status, pw.scan_b, reinterpret_cast<uint64_t*>(d_num_pairs), stream, true,
                          true);
    EmitArgs ea;
    // the record's last float4 holds (., depth, rect01, rect23) in both layouts
    const bool packed = (o.flags & WS_FLAG_PACKED) != 0;
    ea.splats = reinterpret_cast<const float4*>(splats);
    ea.rec_f4 = packed ? 2 : 3;
    ea.rec_tail = packed ? 1 : 2;
    ea.cams = d_cams;
    ea.n_views = n_views;
    ea.list = list;
    ea.offsets = pw.offsets;
    ea.first_entry = pw.first_entry;
    ea.d_nvis = pw.d_nvis;
    ea.d_num_pairs = d_num_pairs;
    ea.d_status = d_status;
    ea.n = std::max<int64_t>(g.n, 1);
    ea.capacity = capacity;
    // keys name cells: tiles, or bins of tiles
    ea.tile_w = o.cell_w();
    ea.tile_h = o.cell_h();
    ea.tw_shift = uint32_t(__builtin_ctz(uint32_t(o.cell_w())));
    ea.th_shift = uint32_t(__builtin_ctz(uint32_t(o.cell_h())));
    ea.tws = uint32_t(__builtin_ctz(uint32_t(o.tile_w)));
    ea.ths = uint32_t(__builtin_ctz(uint32_t(o.tile_h)));
    ea.bxs = uint32_t(__builtin_ctz(uint32_t(o.bin_x)));
    ea.bys = uint32_t(__builtin_ctz(uint32_t(o.bin_y)));
    ea.mask_shift = o.mask_shift;
    ea.keys = keys;
    ea.values = values;
    const bool k32 = (o.flags & WS_FLAG_KEYS32) != 0, mask = o.mask_shift >= 0;
    switch (pw.emit_items) {
        case 2: launch_emit<2>(ea, k32, mask, pw.emit_blocks, stream); break;
        case 4: launch_emit<4>(ea, k32, mask, pw.emit_blocks, stream); break;
        default: launch_emit<8>(ea, k32, mask, pw.emit_blocks, stream); break;
    }
    timing_end(WS_KERNEL_SCAN_EMIT, stream);
    return hipGetLastError();
}

}  // namespace ws
