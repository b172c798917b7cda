// Tile ranges and front-to-back compositing (Eq. 2, Eq. 4).
//
// k_ranges                    [start, end) of every tile's run of pairs in the
//                             tile-sorted key list, written where the tile
//                             changes (the key's cell word: key >> 32, or the
//                             32-bit key itself, without the bins' coverage
//                             mask); the tiles without pairs between two runs
//                             get an empty range at that boundary, so every
//                             tile is written once and no clearing launch is
//                             needed.
// k_render<TW, TH>            one workgroup of TW*TH threads per tile, one
//                             pixel per thread, one 8x8 quadrant per wave.
//                             The tile's splats are staged in LDS in batches
//                             of TW*TH records (each thread gathers one
//                             48-byte record) together with per-quadrant
//                             ballot masks; every wave then walks, front to
//                             back, the staged splats that meet its quadrant.
//                             The workgroup leaves as soon as all its pixels
//                             have stopped.
// k_tile_classes / k_tile_order  (WS_FLAG_ORDERED_RENDER) group the tiles by
//                             the power of two of their pair count and list
//                             them longest first;
// k_render_queue<TW, TH>      persistent workgroups (as many as are resident
//                             at once) take tiles from that list through an
//                             atomic counter until it is exhausted, so the
//                             longest tiles start first and no workgroup
//                             waits for another.  The order in which tiles are
//                             processed does not change any pixel.
// k_expand_bin<K>             (bins larger than one tile, keys carrying the
//                             coverage mask) one workgroup per bin, one wave
//                             per tile of the bin: the waves stream the bin's
//                             run of pairs together and each keeps, in order,
//                             the ids whose coverage bit names its tile,
//                             writing them to a slot of the bin's pair count
//                             reserved for that tile.
// k_expand                    (larger bins, keys without the mask) the same
//                             lists, one workgroup per tile, deciding from
//                             each splat's pixel rectangle.
// The per-(pixel, splat) arithmetic lives in composite.h and is shared with
// the backward pass, so both take exactly the same skip / stop decisions.
#include "composite.h"
#include "ws_internal.h"

namespace ws {
namespace {

// Grid-stride over chunks of 8 x 256 consecutive pairs: every key is loaded
// once (coalesced, all 8 loads of a thread in flight together), its
// predecessor and successor come from the neighbouring lanes (the wave's end
// lanes load theirs).  Tile t's range is [first pair with tile >= t, first
// pair with tile > t): a run's first pair writes its start, its last pair its
// end, and the last pair of a run also writes the empty ranges of the tiles
// between its tile and the next run's (the whole wave writes each such gap,
// so a long gap costs few stores per lane).  Tiles before the first run are
// written by workgroup 0; an empty key list makes every range [0, 0).
constexpr int kRangeThreads = 256;
constexpr int kRangeItems = 8;

__device__ __forceinline__ void fill_empty(uint32_t* ranges, uint32_t lo, uint32_t hi, uint32_t pos, uint32_t first,
                                           uint32_t step) {
    uint2* r = reinterpret_cast<uint2*>(ranges);
    for (uint32_t t = lo + first; t < hi; t += step) r[t] = make_uint2(pos, pos);
}

// The tile (or bin) a key names: the high word of a 64-bit key, a 32-bit key itself.
__device__ __forceinline__ uint32_t cell_of(uint64_t k) { return uint32_t(k >> 32); }
__device__ __forceinline__ uint32_t cell_of(uint32_t k) { return k; }

template <typename K>
__global__ __launch_bounds__(kRangeThreads) void k_ranges(const K* __restrict__ keys, int64_t cap,
                                                          const int64_t* d_n, const int32_t* d_status,
                                                          uint32_t* __restrict__ ranges, int64_t total_tiles,
                                                          uint32_t cell_mask) {
    if (*d_status != 0) return;
    int64_t m = *d_n;
    m = m < cap ? m : cap;
    const uint32_t T = uint32_t(total_tiles);
    // only the cell word of each key is read: the key itself, or the high
    // word of a 64-bit key, as 32-bit loads (the same code for both widths)
    constexpr int64_t S = int64_t(sizeof(K) / 4);
    const uint32_t* __restrict__ cw = reinterpret_cast<const uint32_t*>(keys) + (S - 1);
    if (m == 0) {
        fill_empty(ranges, 0, T, 0, blockIdx.x * kRangeThreads + threadIdx.x, gridDim.x * kRangeThreads);
        return;
    }
    if (blockIdx.x == 0) {  // tiles before the first run
        const uint32_t t0 = cw[0] & cell_mask;
        fill_empty(ranges, 0, t0 < T ? t0 : T, 0, threadIdx.x, kRangeThreads);
    }
    const uint32_t lane = lane_id();
    constexpr int64_t kChunk = int64_t(kRangeThreads) * kRangeItems;
    const int64_t stride = int64_t(gridDim.x) * kChunk;
    for (int64_t base = int64_t(blockIdx.x) * kChunk; base < m; base += stride) {
        // the wave's end lanes also load the neighbour outside the wave
        const int64_t off = lane == 0 ? -1 : (lane == kWave - 1 ? 1 : 0);
        uint32_t t[kRangeItems], edge[kRangeItems];
#pragma unroll
        for (int j = 0; j < kRangeItems; ++j) {
            const int64_t i = base + j * kRangeThreads + threadIdx.x;
            t[j] = i < m ? cw[i * S] : 0xffffffffu;
            const int64_t ie = i + off;
            edge[j] = (off != 0 && ie >= 0 && ie < m) ? cw[ie * S] : 0xffffffffu;
        }
        // the coverage bits are stripped only once every load has been issued
        // (masking inside the loads' conditions made the compiler wait after each)
#pragma unroll
        for (int j = 0; j < kRangeItems; ++j) {
            const int64_t i = base + j * kRangeThreads + threadIdx.x;
            if (i < m) t[j] &= cell_mask;
            const int64_t ie = i + off;
            if (off != 0 && ie >= 0 && ie < m) edge[j] &= cell_mask;
        }
#pragma unroll
        for (int j = 0; j < kRangeItems; ++j) {
            const int64_t i = base + j * kRangeThreads + threadIdx.x;
            uint32_t prev = uint32_t(__shfl_up(int(t[j]), 1, kWave));
            if (lane == 0) prev = edge[j];
            uint32_t next = uint32_t(__shfl_down(int(t[j]), 1, kWave));
            if (lane == kWave - 1) next = edge[j];
            // empty tiles (t, min(next tile, T)) after the last pair of a run
            uint32_t glo = 0, ghi = 0;
            if (i < m) {
                const uint32_t cur = t[j];
                const bool first = i == 0 || prev != cur;
                const bool last = i == m - 1 || next != cur;
                if (cur < T) {  // keys from ws_preprocess never exceed it
                    if (first) ranges[2 * int64_t(cur)] = uint32_t(i);
                    if (last) ranges[2 * int64_t(cur) + 1] = uint32_t(i + 1);
                }
                if (last && cur < T && cur + 1 < T) {
                    glo = cur + 1;
                    ghi = i == m - 1 ? T : (next < T ? next : T);
                }
            }
            uint64_t gaps = __ballot(ghi > glo);
            while (gaps) {
                const int l = __builtin_ctzll(gaps);
                const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(glo), l));
                const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(ghi), l));
                const uint32_t pos = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(i + 1)), l));
                fill_empty(ranges, lo, hi, pos, lane, kWave);
                gaps &= gaps - 1;
            }
        }
    }
}

// ---- per-tile lists from bin lists
//
// A bin of 2^bxs x 2^bys tiles owns the run [bs, be) of the bin-sorted pairs;
// its tile k (row-major inside the bin) writes its list at
// (bs << (bxs + bys)) + k * (be - bs), a slot as long as the bin's run, so the
// slots of all tiles of all bins are disjoint and no count or prefix sum over
// tiles is needed first.  A tile keeps the pairs whose pixel rectangle meets
// it: the same test by which the emission would have listed the splat in that
// tile (the tile range is the pixel range shifted by log2 of the tile size),
// so the list equals the tile's run of pairs under tile keys.  Items are taken
// in list order (item j of thread t is entry c + j * 256 + t) and placed by
// wave ballots and a per-round count in LDS, so the order is preserved.
constexpr int kExpandThreads = 256;
constexpr int kExpandItems = 4;
constexpr int kExpandWaves = kExpandThreads / kWave;

struct ExpandArgs {
    const uint2* splats;  // records of rec_u2 uint2s; uint2 rect_u2 of each is (x0 | x1 << 16, y0 | y1 << 16)
    int32_t rec_u2, rect_u2;
    int64_t n;
    const ws_camera* cams;
    int32_t n_views;
    int32_t tile_w, tile_h;
    uint32_t tws, ths;  // log2 of the tile size
    uint32_t bxs, bys;  // log2 of the bin size in tiles
    int64_t blocks;     // bins << (bxs + bys)
    const void* keys;   // the bin-sorted keys (read where they carry the coverage mask)
    int32_t mask_shift;
    const uint32_t* values;
    const uint32_t* bin_ranges;
    const int32_t* d_status;
    uint32_t* tile_values;
    uint32_t* tile_ranges;
};

__global__ __launch_bounds__(kExpandThreads) void k_expand(ExpandArgs a) {
    __shared__ uint32_t s_cnt[2][kExpandItems][kExpandWaves];
    if (*a.d_status != 0) return;
    // Workgroups are dealt to the 8 XCDs in turn; numbering them XCD-major
    // puts the tiles of one bin (consecutive logical blocks) on one XCD, so
    // that its L2 serves the bin's list to all of them.  The grid is a
    // multiple of 8, so every logical block below 8 * per is produced.
    const uint32_t per = gridDim.x / 8;
    const int64_t L = int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (L >= a.blocks) return;
    const uint32_t kl = a.bxs + a.bys;
    const int64_t bin = L >> kl;
    const uint32_t k = uint32_t(L) & ((1u << kl) - 1u);
    int64_t boff = 0, toff = 0;
    int32_t v = 0, txn = 1, tyn = 1, bxn = 1;
    for (;; ++v) {
        txn = ceil_div(a.cams[v].width, a.tile_w);
        tyn = ceil_div(a.cams[v].height, a.tile_h);
        bxn = (txn + (1 << a.bxs) - 1) >> a.bxs;
        const int64_t nb = int64_t(bxn) * ((tyn + (1 << a.bys) - 1) >> a.bys);
        if (bin < boff + nb || v == a.n_views - 1) break;
        boff += nb;
        toff += int64_t(txn) * tyn;
    }
    const int64_t lb = bin - boff;
    const int32_t by = int32_t(lb / bxn), bx = int32_t(lb - int64_t(by) * bxn);
    const int32_t tx = (bx << a.bxs) + int32_t(k & ((1u << a.bxs) - 1u));
    const int32_t ty = (by << a.bys) + int32_t(k >> a.bxs);
    if (tx >= txn || ty >= tyn) return;  // bins on the right / bottom edge hold fewer tiles
    const int64_t tile = toff + int64_t(ty) * txn + tx;
    const uint32_t bs = a.bin_ranges[2 * bin], be = a.bin_ranges[2 * bin + 1];
    const uint32_t base = (bs << kl) + k * (be - bs);
    const uint2* vs = a.splats + int64_t(v) * a.n * a.rec_u2;
    const uint32_t lane = lane_id();
    const int wave = threadIdx.x / kWave;
    uint32_t count = 0;
    int buf = 0;
    for (uint32_t c = bs; c < be; c += kExpandThreads * kExpandItems) {
        uint32_t id[kExpandItems];
        bool keep[kExpandItems];
#pragma unroll
        for (int j = 0; j < kExpandItems; ++j) {
            const uint32_t idx = c + uint32_t(j * kExpandThreads) + threadIdx.x;
            id[j] = idx < be ? a.values[idx] : 0xffffffffu;
        }
#pragma unroll
        for (int j = 0; j < kExpandItems; ++j) {
            keep[j] = false;
            if (id[j] < uint64_t(a.n)) {
                // the record's rectangle words: x0 | x1 << 16, y0 | y1 << 16
                const uint2 r = vs[int64_t(id[j]) * a.rec_u2 + a.rect_u2];
                const int32_t tx0 = int32_t((r.x & 0xffffu) >> a.tws), tx1 = int32_t((r.x >> 16) >> a.tws);
                const int32_t ty0 = int32_t((r.y & 0xffffu) >> a.ths), ty1 = int32_t((r.y >> 16) >> a.ths);
                keep[j] = tx0 <= tx && tx <= tx1 && ty0 <= ty && ty <= ty1;
            }
        }
        uint32_t below[kExpandItems];
#pragma unroll
        for (int j = 0; j < kExpandItems; ++j) {
            const uint64_t m = __builtin_amdgcn_ballot_w64(keep[j]);
            below[j] = lanes_below(m);
            if (lane == 0) s_cnt[buf][j][wave] = uint32_t(__builtin_popcountll(m));
        }
        __syncthreads();
        uint32_t pos = count;
#pragma unroll
        for (int j = 0; j < kExpandItems; ++j) {
            uint32_t wpre = 0, tot = 0;
#pragma unroll
            for (int w = 0; w < kExpandWaves; ++w) {
                const uint32_t cw = s_cnt[buf][j][w];
                wpre += w < wave ? cw : 0u;
                tot += cw;
            }
            if (keep[j]) a.tile_values[base + pos + wpre + below[j]] = id[j];
            pos += tot;
        }
        count = pos;
        buf ^= 1;  // the next round writes the other half: one barrier per round suffices
    }
    if (threadIdx.x == 0) {
        a.tile_ranges[2 * tile] = base;
        a.tile_ranges[2 * tile + 1] = base + count;
    }
}

// One workgroup per bin of a view (the bin ids of all views in order), wave w
// handling tile w of the bin (row-major inside the bin); the tile's slot and
// list are those of k_expand.  Each wave reads the bin's keys and ids (the
// waves of a workgroup read the same addresses, so the bin's run comes from
// HBM about once), keeps the pairs whose coverage bit w is set and compacts
// them in order with a ballot per item: no LDS and no barrier.  Waves of tiles
// past the view's right or bottom edge leave at once.
constexpr int kExpandBinItems = 16;

template <typename K>
__global__ __launch_bounds__(1024) void k_expand_bin(ExpandArgs a, int64_t bins) {
    if (*a.d_status != 0) return;
    const int64_t bin = blockIdx.x;
    if (bin >= bins) return;
    const uint32_t k = threadIdx.x / kWave;  // tile of the bin
    const uint32_t kl = a.bxs + a.bys;
    int64_t boff = 0, toff = 0;
    int32_t v = 0, txn = 1, tyn = 1, bxn = 1;
    for (;; ++v) {
        txn = ceil_div(a.cams[v].width, a.tile_w);
        tyn = ceil_div(a.cams[v].height, a.tile_h);
        bxn = (txn + (1 << a.bxs) - 1) >> a.bxs;
        const int64_t nb = int64_t(bxn) * ((tyn + (1 << a.bys) - 1) >> a.bys);
        if (bin < boff + nb || v == a.n_views - 1) break;
        boff += nb;
        toff += int64_t(txn) * tyn;
    }
    const int64_t lb = bin - boff;
    const int32_t by = int32_t(lb / bxn), bx = int32_t(lb - int64_t(by) * bxn);
    const int32_t tx = (bx << a.bxs) + int32_t(k & ((1u << a.bxs) - 1u));
    const int32_t ty = (by << a.bys) + int32_t(k >> a.bxs);
    if (tx >= txn || ty >= tyn) return;  // bins on the right / bottom edge hold fewer tiles
    const int64_t tile = toff + int64_t(ty) * txn + tx;
    const uint32_t bs = a.bin_ranges[2 * bin], be = a.bin_ranges[2 * bin + 1];
    const uint32_t base = (bs << kl) + k * (be - bs);
    const K* keys = static_cast<const K*>(a.keys);
    const uint32_t lane = lane_id();
    uint32_t count = 0;
    for (uint32_t c = bs; c < be; c += kWave * kExpandBinItems) {
        uint32_t id[kExpandBinItems], cov[kExpandBinItems];
        // every load of the round in flight before the first use
#pragma unroll
        for (int j = 0; j < kExpandBinItems; ++j) {
            const uint32_t idx = c + uint32_t(j * kWave) + lane;
            const uint32_t ic = idx < be ? idx : be - 1;
            id[j] = a.values[ic];
            cov[j] = cell_of(keys[ic]);
        }
#pragma unroll
        for (int j = 0; j < kExpandBinItems; ++j) {
            const uint32_t idx = c + uint32_t(j * kWave) + lane;
            const bool keep = idx < be && id[j] < uint64_t(a.n) && (((cov[j] >> a.mask_shift) >> k) & 1u) != 0u;
            const uint64_t m = __builtin_amdgcn_ballot_w64(keep);
            if (keep) a.tile_values[base + count + lanes_below(m)] = id[j];
            count += uint32_t(__builtin_popcountll(m));
        }
    }
    if (lane == 0) {
        a.tile_ranges[2 * tile] = base;
        a.tile_ranges[2 * tile + 1] = base + count;
    }
}

struct RenderArgs {
    const ws_splat* splats;
    int64_t n;
    const ws_camera* cams;
    int32_t n_views;
    int64_t total_tiles;
    const uint32_t* values;
    const uint32_t* ranges;
    float* images;
    const int32_t* d_status;
    KOpts o;
};

// Staging of one batch: thread t stages list entry b0 + t (if any) and the
// quadrant masks of the batch are formed; the caller synchronises afterwards.
template <int TW, int TH>
__device__ __forceinline__ void stage_batch(const RenderArgs& a, const ws_splat* vsplats, uint32_t b0, uint32_t end,
                                            int x0, int y0, float log2_amin, StagedSplat* s_batch,
                                            uint64_t* s_masks) {
    const uint32_t idx = b0 + threadIdx.x;
    StagedSplat s = empty_splat();
    bool valid = false;
    if (idx < end) {
        const uint32_t id = a.values[idx];
        if (id < uint64_t(a.n)) {
            s = (a.o.flags & WS_FLAG_PACKED) ? stage_splat_packed(reinterpret_cast<const float4*>(vsplats), id)
                                             : stage_splat(vsplats, id);
            valid = true;
        }
        s_batch[threadIdx.x] = s;
    }
    stage_quadrant_masks<TW, TH>(s, valid, x0, y0, log2_amin, s_masks);
}

// Composites global tile g into the images (RECT: see blend_one).
template <int TW, int TH, bool RECT>
__device__ __forceinline__ void render_tile(const RenderArgs& a, int64_t g, StagedSplat* s_batch, uint64_t* s_masks) {
    constexpr int NT = TW * TH, NW = NT / kWave;
    const TileInfo ti = locate_tile(a.cams, a.n_views, g, TW, TH);
    int px, py;
    quadrant_pixel<TW>(ti.x0, ti.y0, &px, &py);
    const bool inside = px < ti.W && py < ti.H;
    const uint32_t start = a.ranges[2 * g], end = a.ranges[2 * g + 1];
    // the view's records: 48-byte ws_splat, or 32-byte ws_splat_packed (addressed in float4s)
    const ws_splat* vsplats = (a.o.flags & WS_FLAG_PACKED)
                                  ? reinterpret_cast<const ws_splat*>(reinterpret_cast<const float4*>(a.splats) +
                                                                      2 * int64_t(ti.view) * a.n)
                                  : a.splats + int64_t(ti.view) * a.n;
    const uint64_t* my_masks = s_masks + (threadIdx.x / kWave) * NW;
    PixelState ps;
    ps.init(px, py);
    uint64_t active = wave_ballot(inside);  // lanes whose pixel is still compositing
    const BlendConsts bk(a.o);
    for (uint32_t b0 = start; b0 < end; b0 += NT) {
        if (__syncthreads_count(!lane_in(active)) == NT) break;
        stage_batch<TW, TH>(a, vsplats, b0, end, ti.x0, ti.y0, bk.log2_amin, s_batch, s_masks);
        __syncthreads();
        composite_batch<NW, RECT>(ps, active, s_batch, my_masks, int32_t(b0 - start), bk);
    }
    if (inside) {
        float* img = a.images + ti.img_off;
        const int64_t plane = int64_t(ti.W) * ti.H;
        const int64_t p = int64_t(py) * ti.W + px;
        img[p] = ps.c[0] + ps.T * a.o.bg[0];
        img[plane + p] = ps.c[1] + ps.T * a.o.bg[1];
        img[2 * plane + p] = ps.c[2] + ps.T * a.o.bg[2];
    }
}

template <int TW, int TH, bool RECT>
__global__ __launch_bounds__(TW * TH) void k_render(RenderArgs a) {
    constexpr int NW = TW * TH / kWave;
    __shared__ StagedSplat s_batch[TW * TH];
    __shared__ uint64_t s_masks[NW * NW];
    if (*a.d_status != 0) return;
    render_tile<TW, TH, RECT>(a, blockIdx.x, s_batch, s_masks);
}

// ---- ordered, persistent render

constexpr int kClasses = 33;  // 0: empty tile; c >= 1: pair count in [2^(c-1), 2^c)

__device__ __forceinline__ int tile_class(const uint32_t* ranges, int64_t t) {
    const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
    return len ? 32 - __builtin_clz(len) : 0;
}

// Tile counts per class (counters zeroed beforehand).
__global__ __launch_bounds__(256) void k_tile_classes(const uint32_t* ranges, int64_t total_tiles,
                                                      const int32_t* d_status, uint32_t* hist) {
    __shared__ uint32_t s_h[kClasses];
    if (*d_status != 0) return;
    for (int i = threadIdx.x; i < kClasses; i += 256) s_h[i] = 0;
    __syncthreads();
    const int64_t stride = int64_t(gridDim.x) * 256;
    for (int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x; t < total_tiles; t += stride)
        atomicAdd(&s_h[tile_class(ranges, t)], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < kClasses; i += 256)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

// order[] lists the tiles by descending class (any order inside a class).
__global__ __launch_bounds__(256) void k_tile_order(const uint32_t* ranges, int64_t total_tiles,
                                                    const int32_t* d_status, const uint32_t* hist,
                                                    uint32_t* cursor, uint32_t* order) {
    __shared__ uint32_t s_base[kClasses];
    if (*d_status != 0) return;
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int c = kClasses - 1; c >= 0; --c) {
            s_base[c] = run;
            run += hist[c];
        }
    }
    __syncthreads();
    const int64_t stride = int64_t(gridDim.x) * 256;
    for (int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x; t < total_tiles; t += stride) {
        const int c = tile_class(ranges, t);
        const uint32_t pos = s_base[c] + atomicAdd(&cursor[c], 1u);
        if (int64_t(pos) < total_tiles) order[pos] = uint32_t(t);  // always true for consistent counts
    }
}

// Every workgroup takes list positions from *queue until they run past the
// end; each take advances the counter, so every workgroup leaves.
template <int TW, int TH, bool RECT>
__global__ __launch_bounds__(TW * TH) void k_render_queue(RenderArgs a, const uint32_t* order, uint32_t* queue) {
    constexpr int NW = TW * TH / kWave;
    __shared__ StagedSplat s_batch[TW * TH];
    __shared__ uint64_t s_masks[NW * NW];
    __shared__ uint32_t s_q;
    if (*a.d_status != 0) return;
    while (true) {
        if (threadIdx.x == 0) s_q = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t q = s_q;
        __syncthreads();
        if (int64_t(q) >= a.total_tiles) break;
        render_tile<TW, TH, RECT>(a, order[q], s_batch, s_masks);
    }
}

struct OrderWs {
    uint32_t* order;   // [total_tiles]
    uint32_t* hist;    // [kClasses]
    uint32_t* cursor;  // [kClasses]
    uint32_t* queue;   // [1]
};

size_t order_ws(void* ws, int64_t total_tiles, OrderWs* out) {
    char* base = static_cast<char*>(ws);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* ptr = base ? base + off : nullptr;
        off += align_up(bytes);
        return ptr;
    };
    OrderWs w;
    w.order = reinterpret_cast<uint32_t*>(take(size_t(std::max<int64_t>(total_tiles, 1)) * 4));
    w.hist = reinterpret_cast<uint32_t*>(take((2 * kClasses + 1) * 4));
    w.cursor = w.hist ? w.hist + kClasses : nullptr;
    w.queue = w.hist ? w.hist + 2 * kClasses : nullptr;
    if (out) *out = w;
    return off;
}

__global__ void k_order_clear(uint32_t* words, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) words[i] = 0;
}

// Resident workgroups of k_render_queue on the current device (cached per device).
template <int TW, int TH, bool RECT>
uint32_t persistent_grid() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_render_queue<TW, TH, RECT>, TW * TH, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
        cached[dev] = per_cu * cus;
    }
    return uint32_t(cached[dev]);
}

void launch_ranges(const KOpts& o, const void* keys, int64_t capacity, const int64_t* d_num_pairs,
                   const int32_t* d_status, uint32_t* ranges, int64_t cells, uint32_t grid, hipStream_t stream) {
    if (o.flags & WS_FLAG_KEYS32)
        hipLaunchKernelGGL(k_ranges<uint32_t>, dim3(grid), dim3(kRangeThreads), 0, stream,
                           static_cast<const uint32_t*>(keys), capacity, d_num_pairs, d_status, ranges, cells,
                           o.cell_mask());
    else
        hipLaunchKernelGGL(k_ranges<uint64_t>, dim3(grid), dim3(kRangeThreads), 0, stream,
                           static_cast<const uint64_t*>(keys), capacity, d_num_pairs, d_status, ranges, cells,
                           o.cell_mask());
}

template <int TW, int TH, bool RECT>
void launch_render_rt(const RenderArgs& ra, const OrderWs* ow, hipStream_t stream) {
    if (!ow) {
        hipLaunchKernelGGL((k_render<TW, TH, RECT>), dim3(uint32_t(ra.total_tiles)), dim3(TW * TH), 0, stream, ra);
        return;
    }
    const uint32_t grid = uint32_t(std::min<int64_t>(persistent_grid<TW, TH, RECT>(), ra.total_tiles));
    hipLaunchKernelGGL((k_render_queue<TW, TH, RECT>), dim3(grid), dim3(TW * TH), 0, stream, ra,
                       static_cast<const uint32_t*>(ow->order), ow->queue);
}

// The rectangle test is needed only where the ellipse the render evaluates
// may reach beyond the rectangle: the fixed 3-sigma extent, and packed records
// (the rectangle bounds the ellipse before its axes are rounded to fp16).
template <int TW, int TH>
void launch_render_t(const RenderArgs& ra, const OrderWs* ow, hipStream_t stream) {
    if (ra.o.flags & (WS_FLAG_FIXED_3SIGMA | WS_FLAG_PACKED)) launch_render_rt<TW, TH, true>(ra, ow, stream);
    else launch_render_rt<TW, TH, false>(ra, ow, stream);
}

}  // namespace

size_t expand_workspace(int64_t total_bins) { return align_up(size_t(std::max<int64_t>(total_bins, 1)) * 8); }

hipError_t launch_expand(const ws_splat* splats, int64_t n, const ws_camera* d_cams, int32_t n_views,
                         int64_t total_bins, const KOpts& o, const void* keys, const uint32_t* values,
                         int64_t capacity, const int64_t* d_num_pairs, const int32_t* d_status,
                         uint32_t* tile_values, uint32_t* tile_ranges, void* ws, hipStream_t stream) {
    uint32_t* bin_ranges = static_cast<uint32_t*>(ws);
    timing_begin(WS_KERNEL_RANGES, stream);
    const int64_t rchunk = int64_t(kRangeThreads) * kRangeItems;
    const uint32_t rgrid = uint32_t(std::min<int64_t>(std::max<int64_t>((capacity + rchunk - 1) / rchunk, 1), 4096));
    launch_ranges(o, keys, capacity, d_num_pairs, d_status, bin_ranges, total_bins, rgrid, stream);
    ExpandArgs ea;
    const bool packed = (o.flags & WS_FLAG_PACKED) != 0;
    ea.splats = reinterpret_cast<const uint2*>(splats);
    ea.rec_u2 = packed ? 4 : 6;   // 32- or 48-byte records
    ea.rect_u2 = packed ? 3 : 5;  // words 6-7 or 10-11
    ea.n = std::max<int64_t>(n, 1);
    ea.cams = d_cams;
    ea.n_views = n_views;
    ea.tile_w = o.tile_w;
    ea.tile_h = o.tile_h;
    ea.tws = uint32_t(__builtin_ctz(uint32_t(o.tile_w)));
    ea.ths = uint32_t(__builtin_ctz(uint32_t(o.tile_h)));
    ea.bxs = uint32_t(__builtin_ctz(uint32_t(o.bin_x)));
    ea.bys = uint32_t(__builtin_ctz(uint32_t(o.bin_y)));
    ea.blocks = total_bins << (ea.bxs + ea.bys);
    ea.keys = keys;
    ea.mask_shift = o.mask_shift;
    ea.values = values;
    ea.bin_ranges = bin_ranges;
    ea.d_status = d_status;
    ea.tile_values = tile_values;
    ea.tile_ranges = tile_ranges;
    const uint32_t grid = uint32_t((ea.blocks + 7) / 8 * 8);
    const bool k32 = (o.flags & WS_FLAG_KEYS32) != 0;
    if (o.mask_shift >= 0) {  // one workgroup per bin, one wave per tile of the bin (at most 16 tiles)
        const uint32_t threads = uint32_t(kWave << (ea.bxs + ea.bys));
        if (total_bins > 0) {
            if (k32)
                hipLaunchKernelGGL(k_expand_bin<uint32_t>, dim3(uint32_t(total_bins)), dim3(threads), 0, stream, ea,
                                   total_bins);
            else
                hipLaunchKernelGGL(k_expand_bin<uint64_t>, dim3(uint32_t(total_bins)), dim3(threads), 0, stream, ea,
                                   total_bins);
        }
    } else if (grid > 0) {
        hipLaunchKernelGGL(k_expand, dim3(grid), dim3(kExpandThreads), 0, stream, ea);
    }
    timing_end(WS_KERNEL_RANGES, stream);
    return hipGetLastError();
}

size_t render_workspace(int64_t total_tiles, const KOpts& o) {
    if (o.flags & WS_FLAG_ORDERED_RENDER) return order_ws(nullptr, total_tiles, nullptr);
    return align_up(64);
}

hipError_t launch_render(const ws_splat* splats, int64_t n, const ws_camera* d_cams, int32_t n_views,
                         int64_t total_tiles, const KOpts& o, const void* keys, const uint32_t* values,
                         int64_t capacity, const int64_t* d_num_pairs, const int32_t* d_status,
                         uint32_t* tile_ranges, float* images, void* ws, hipStream_t stream) {
    if (keys) {  // otherwise the ranges are given (ws_expand_bins)
        timing_begin(WS_KERNEL_RANGES, stream);
        const int64_t rchunk = int64_t(kRangeThreads) * kRangeItems;
        const uint32_t rgrid =
            uint32_t(std::min<int64_t>(std::max<int64_t>((capacity + rchunk - 1) / rchunk, 1), 4096));
        launch_ranges(o, keys, capacity, d_num_pairs, d_status, tile_ranges, total_tiles, rgrid, stream);
        timing_end(WS_KERNEL_RANGES, stream);
    }
    if (total_tiles == 0) return hipGetLastError();
    RenderArgs ra;
    ra.splats = splats;
    ra.n = n;
    ra.cams = d_cams;
    ra.n_views = n_views;
    ra.total_tiles = total_tiles;
    ra.values = values;
    ra.ranges = tile_ranges;
    ra.images = images;
    ra.d_status = d_status;
    ra.o = o;
    OrderWs ow;
    const bool ordered = (o.flags & WS_FLAG_ORDERED_RENDER) != 0;
    timing_begin(WS_KERNEL_RENDER, stream);
    if (ordered) {
        order_ws(ws, total_tiles, &ow);
        const uint32_t ogrid = uint32_t(std::min<int64_t>((total_tiles + 255) / 256, 1024));
        hipLaunchKernelGGL(k_order_clear, dim3(1), dim3(128), 0, stream, ow.hist, 2 * kClasses + 1);
        hipLaunchKernelGGL(k_tile_classes, dim3(ogrid), dim3(256), 0, stream, static_cast<const uint32_t*>(tile_ranges),
                           total_tiles, d_status, ow.hist);
        hipLaunchKernelGGL(k_tile_order, dim3(ogrid), dim3(256), 0, stream, static_cast<const uint32_t*>(tile_ranges),
                           total_tiles, d_status, static_cast<const uint32_t*>(ow.hist), ow.cursor, ow.order);
    }
    const OrderWs* owp = ordered ? &ow : nullptr;
    if (o.tile_w == 16 && o.tile_h == 16) launch_render_t<16, 16>(ra, owp, stream);
    else if (o.tile_w == 8 && o.tile_h == 8) launch_render_t<8, 8>(ra, owp, stream);
    else if (o.tile_w == 16 && o.tile_h == 8) launch_render_t<16, 8>(ra, owp, stream);
    else launch_render_t<32, 16>(ra, owp, stream);
    timing_end(WS_KERNEL_RENDER, stream);
    return hipGetLastError();
}

}  // namespace ws
