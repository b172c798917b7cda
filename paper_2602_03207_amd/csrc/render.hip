// Tile ranges and front-to-back compositing (Eq. 2, Eq. 4).
//
// k_ranges_clear / k_ranges   [start, end) of every tile's run of pairs in the
//                             tile-sorted key list (boundary where key >> 32
//                             changes); tiles without pairs keep [0, 0).
// k_render<TW, TH>            one workgroup of TW*TH threads per tile, one
//                             pixel per thread.  The tile's splats are staged
//                             in LDS in batches of TW*TH records (each thread
//                             gathers one 48-byte record); every lane then
//                             walks the batch front to back.  The workgroup
//                             leaves as soon as all its pixels have stopped.
// The per-(pixel, splat) arithmetic lives in composite.h and is shared with
// the backward pass, so both take exactly the same skip / stop decisions.
#include "composite.h"
#include "ws_internal.h"

namespace ws {
namespace {

__global__ void k_ranges_clear(uint32_t* ranges, int64_t words, uint32_t* counter) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < words; i += stride) ranges[i] = 0;
    if (counter && blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
}

__global__ void k_ranges(const uint64_t* __restrict__ keys, int64_t cap, const int64_t* d_n,
                         const int32_t* d_status, uint32_t* __restrict__ ranges, int64_t total_tiles) {
    if (*d_status != 0) return;
    int64_t m = *d_n;
    m = m < cap ? m : cap;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += stride) {
        const uint32_t t = uint32_t(keys[i] >> 32);
        if (int64_t(t) >= total_tiles) continue;  // keys from ws_preprocess never exceed it
        if (i == 0 || uint32_t(keys[i - 1] >> 32) != t) ranges[2 * int64_t(t)] = uint32_t(i);
        if (i == m - 1 || uint32_t(keys[i + 1] >> 32) != t) ranges[2 * int64_t(t) + 1] = uint32_t(i + 1);
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

template <int TW, int TH>
__global__ __launch_bounds__(TW * TH) void k_render(RenderArgs a) {
    constexpr int NT = TW * TH;
    __shared__ StagedSplat s_batch[NT];
    if (*a.d_status != 0) return;
    const int64_t g = blockIdx.x;
    TileInfo ti = locate_tile(a.cams, a.n_views, g, TW, TH);
    const int px = ti.x0 + int(threadIdx.x % TW), py = ti.y0 + int(threadIdx.x / TW);
    const bool inside = px < ti.W && py < ti.H;
    const uint32_t start = a.ranges[2 * g], end = a.ranges[2 * g + 1];
    const ws_splat* vsplats = a.splats + int64_t(ti.view) * a.n;
    PixelState ps;
    ps.init(px, py, !inside);
    for (uint32_t b0 = start; b0 < end; b0 += NT) {
        if (__syncthreads_count(ps.done) == NT) break;
        const uint32_t idx = b0 + threadIdx.x;
        if (idx < end) {
            const uint32_t id = a.values[idx];
            s_batch[threadIdx.x] = id < uint64_t(a.n) ? stage_splat(vsplats, id) : empty_splat();
        }
        __syncthreads();
        composite_batch(ps, s_batch, int(min<uint32_t>(NT, end - b0)), int32_t(b0 - start), a.o);
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

template <int TW, int TH>
void launch_render_t(const RenderArgs& ra, hipStream_t stream) {
    hipLaunchKernelGGL((k_render<TW, TH>), dim3(uint32_t(ra.total_tiles)), dim3(TW * TH), 0, stream, ra);
}

}  // namespace

size_t render_workspace(int64_t total_tiles, const KOpts& o) {
    (void)total_tiles;
    (void)o;
    return align_up(64);
}

hipError_t launch_render(const ws_splat* splats, int64_t n, const ws_camera* d_cams, int32_t n_views,
                         int64_t total_tiles, const KOpts& o, const uint64_t* keys, const uint32_t* values,
                         int64_t capacity, const int64_t* d_num_pairs, const int32_t* d_status,
                         uint32_t* tile_ranges, float* images, void* ws, hipStream_t stream) {
    (void)ws;
    const int64_t words = 2 * total_tiles;
    const uint32_t cgrid = uint32_t(std::min<int64_t>(std::max<int64_t>((words + 255) / 256, 1), 4096));
    timing_begin(WS_KERNEL_RANGES, stream);
    hipLaunchKernelGGL(k_ranges_clear, dim3(cgrid), dim3(256), 0, stream, tile_ranges, words, (uint32_t*)nullptr);
    hipLaunchKernelGGL(k_ranges, dim3(2048), dim3(256), 0, stream, keys, capacity, d_num_pairs, d_status,
                       tile_ranges, total_tiles);
    timing_end(WS_KERNEL_RANGES, stream);
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
    timing_begin(WS_KERNEL_RENDER, stream);
    if (o.tile_w == 16 && o.tile_h == 16) launch_render_t<16, 16>(ra, stream);
    else if (o.tile_w == 8 && o.tile_h == 8) launch_render_t<8, 8>(ra, stream);
    else if (o.tile_w == 16 && o.tile_h == 8) launch_render_t<16, 8>(ra, stream);
    else launch_render_t<32, 16>(ra, stream);
    timing_end(WS_KERNEL_RENDER, stream);
    return hipGetLastError();
}

}  // namespace ws
