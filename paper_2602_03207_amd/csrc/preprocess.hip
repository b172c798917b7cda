// Pre-processing stage (Sec. 3.2) and key emission.
//
// k_preprocess   one thread per (view, Gaussian): opacity cull, projection,
//                bounding-box cull, SH colour; writes the 48-byte splat
//                record of visible splats and tiles_touched of every splat.
// k_scan_emit    one pass over tiles_touched: exclusive prefix sum across the
//                device (decoupled look-back over workgroup aggregates, wait
//                bounded), then each workgroup writes its own pairs
//                (key = tile << 32 | depth bits, value = Gaussian id) with
//                coalesced stores, load-balanced over the pairs rather than
//                over the splats.
#include "project.h"
#include "ws_internal.h"

namespace ws {
namespace {

constexpr int kPreThreads = 256;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;  // entries per workgroup
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagInc = 2ull << 62;
constexpr uint64_t kValueMask = (1ull << 62) - 1;

struct PreprocessWs {
    uint64_t* scan_status;  // [n_blocks]
    uint32_t* ticket;       // [1]
    int64_t n_blocks;
};

PreprocessWs carve(void* ws, int64_t n, int32_t n_views) {
    PreprocessWs p;
    const int64_t total = n * n_views;
    p.n_blocks = (total + kScanTile - 1) / kScanTile;
    char* base = static_cast<char*>(ws);
    p.scan_status = reinterpret_cast<uint64_t*>(base);
    base += align_up(size_t(std::max<int64_t>(p.n_blocks, 1)) * sizeof(uint64_t));
    p.ticket = reinterpret_cast<uint32_t*>(base);
    return p;
}

template <int DEG>
__global__ __launch_bounds__(kPreThreads) void k_preprocess(GaussPtrs g, const ws_camera* __restrict__ cams, KOpts o,
                                                           ws_splat* __restrict__ splats,
                                                           uint32_t* __restrict__ tiles_touched, PreprocessWs pw) {
    const int32_t v = blockIdx.y;
    const int64_t i = int64_t(blockIdx.x) * kPreThreads + threadIdx.x;
    // clear the emission look-back state for the kernel that follows
    const int64_t flat = (int64_t(blockIdx.y) * gridDim.x + blockIdx.x) * kPreThreads + threadIdx.x;
    if (flat < (pw.n_blocks > 0 ? pw.n_blocks : 1)) pw.scan_status[flat] = 0;
    if (flat == 0) *pw.ticket = 0;
    if (i >= g.n) return;
    const ws_camera& cam = cams[v];
    ProjState st;
    const bool vis = compute_projection<DEG>(g, i, cam, o, st);
    const int64_t vi = int64_t(v) * g.n + i;
    tiles_touched[vi] = vis ? st.tiles : 0u;
    if (!vis) return;
    float4* rec = reinterpret_cast<float4*>(splats + vi);
    const uint32_t r01 = uint32_t(st.rect[0]) | (uint32_t(st.rect[1]) << 16);
    const uint32_t r23 = uint32_t(st.rect[2]) | (uint32_t(st.rect[3]) << 16);
    rec[0] = make_float4(st.u, st.v, st.A, st.B);
    rec[1] = make_float4(st.C, st.sigma, st.rgb[0], st.rgb[1]);
    rec[2] = make_float4(st.rgb[2], st.z32, __uint_as_float(r01), __uint_as_float(r23));
}

struct EmitArgs {
    const uint32_t* tiles_touched;
    const ws_splat* splats;
    const ws_camera* cams;
    int32_t n_views;
    int64_t n;
    int64_t total;  // n * n_views
    int32_t tile_w, tile_h;
    uint64_t* keys;
    uint32_t* values;
    int64_t capacity;
    int64_t* d_num_pairs;
    int32_t* d_status;
    int64_t n_launched;  // number of emission blocks launched (>= 1)
};

__global__ __launch_bounds__(kScanThreads) void k_scan_emit(EmitArgs a, PreprocessWs pw) {
    __shared__ uint32_t s_block;
    __shared__ uint64_t s_excl;
    __shared__ uint32_t s_scan[kScanThreads / kWave + 1];
    __shared__ uint32_t s_incl[kScanTile];   // inclusive prefix of pair counts inside the block
    __shared__ uint32_t s_gid[kScanTile];    // Gaussian id
    __shared__ uint32_t s_depth[kScanTile];  // fp32 depth bits
    __shared__ uint32_t s_trect[kScanTile * 2];  // tile rect (tx0 | tx1 << 16, ty0 | ty1 << 16)
    __shared__ uint32_t s_tbase[kScanTile];  // tile id offset of the entry's view
    __shared__ uint32_t s_tilesx[kScanTile];

    if (threadIdx.x == 0) s_block = atomicAdd(pw.ticket, 1u);
    __syncthreads();
    const int64_t blk = s_block;
    const int64_t base = blk * kScanTile;
    // blocked arrangement: thread t owns entries base + 4t .. 4t + 3
    uint32_t cnt[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t idx = base + threadIdx.x * kScanItems + j;
        cnt[j] = idx < a.total ? a.tiles_touched[idx] : 0u;
        sum += cnt[j];
    }
    uint32_t block_total;
    const uint32_t texcl = block_exclusive_scan<kScanThreads>(sum, s_scan, &block_total);

    // ---- decoupled look-back over the preceding blocks (wave 0)
    if (threadIdx.x < kWave) {
        const uint32_t lane = threadIdx.x;
        uint64_t excl = 0;
        if (blk == 0) {
            if (lane == 0) store_agent(&pw.scan_status[0], kFlagInc | block_total);
        } else {
            if (lane == 0) store_agent(&pw.scan_status[blk], kFlagAgg | block_total);
            int64_t look = blk - 1;
            uint32_t spins = 0;
            bool failed = false;
            while (true) {
                const int64_t idx = look - int64_t(lane);
                uint64_t s = idx >= 0 ? load_agent(&pw.scan_status[idx]) : kFlagInc;
                while (__ballot((s >> 62) == 0) != 0) {
                    if (++spins > kSpinLimit) { failed = true; break; }
                    __builtin_amdgcn_s_sleep(1);
                    if ((s >> 62) == 0) s = load_agent(&pw.scan_status[idx]);
                }
                if (failed) break;
                const uint64_t inc_mask = __ballot((s >> 62) == 2);
                if (inc_mask != 0) {
                    const uint32_t first = __builtin_ctzll(inc_mask);
                    const uint64_t part = lane <= first ? (s & kValueMask) : 0ull;
                    excl += wave_sum(part);
                    break;
                }
                excl += wave_sum(s & kValueMask);
                look -= kWave;
            }
            if (failed) {
                if (lane == 0) atomicExch(a.d_status, int32_t(WS_ERR_SPIN_LIMIT));
                excl = 0;
            }
            if (lane == 0) store_agent(&pw.scan_status[blk], kFlagInc | (excl + block_total));
        }
        if (lane == 0) s_excl = excl;
    }
    // ---- per-entry data for the emission
    uint32_t run = texcl;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int e = threadIdx.x * kScanItems + j;
        const int64_t idx = base + e;
        run += cnt[j];
        s_incl[e] = run;
        if (cnt[j] != 0) {
            const int64_t view = idx / a.n;
            const int64_t gid = idx - view * a.n;
            const float4 r2 = reinterpret_cast<const float4*>(a.splats + idx)[2];
            const uint32_t r01 = __float_as_uint(r2.z), r23 = __float_as_uint(r2.w);
            const uint32_t tx0 = (r01 & 0xffffu) / uint32_t(a.tile_w), tx1 = (r01 >> 16) / uint32_t(a.tile_w);
            const uint32_t ty0 = (r23 & 0xffffu) / uint32_t(a.tile_h), ty1 = (r23 >> 16) / uint32_t(a.tile_h);
            int64_t toff, ioff;
            view_offsets(a.cams, int32_t(view), a.tile_w, a.tile_h, &toff, &ioff);
            s_gid[e] = uint32_t(gid);
            s_depth[e] = __float_as_uint(r2.y);
            s_trect[2 * e] = tx0 | (tx1 << 16);
            s_trect[2 * e + 1] = ty0 | (ty1 << 16);
            s_tbase[e] = uint32_t(toff);
            s_tilesx[e] = uint32_t(ceil_div(a.cams[view].width, a.tile_w));
        }
    }
    __syncthreads();
    const uint64_t excl = s_excl;
    if (blk == a.n_launched - 1 && threadIdx.x == 0) {
        const uint64_t m = excl + block_total;
        *a.d_num_pairs = int64_t(m);
        if (int64_t(m) > a.capacity) atomicMax(a.d_status, int32_t(WS_ERR_CAPACITY));
    }
    // ---- emission: pair j of this block belongs to the first entry e with s_incl[e] > j
    for (uint32_t j = threadIdx.x; j < block_total; j += kScanThreads) {
        int lo = 0, hi = kScanTile - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_incl[mid] > j) hi = mid; else lo = mid + 1;
        }
        const int e = lo;
        const uint32_t start = e > 0 ? s_incl[e - 1] : 0u;
        const uint32_t k = j - start;
        const uint32_t xr = s_trect[2 * e], yr = s_trect[2 * e + 1];
        const uint32_t tx0 = xr & 0xffffu, tx1 = xr >> 16, ty0 = yr & 0xffffu;
        const uint32_t w = tx1 - tx0 + 1;
        const uint32_t row = k / w, col = k - row * w;
        const uint64_t tile = uint64_t(s_tbase[e]) + uint64_t(ty0 + row) * s_tilesx[e] + (tx0 + col);
        const uint64_t pos = excl + j;
        if (int64_t(pos) < a.capacity) {
            a.keys[pos] = (tile << 32) | s_depth[e];
            a.values[pos] = s_gid[e];
        }
    }
}

}  // namespace

size_t preprocess_workspace(int64_t n, int32_t n_views) {
    const int64_t blocks = std::max<int64_t>((n * n_views + kScanTile - 1) / kScanTile, 1);
    return align_up(size_t(blocks) * sizeof(uint64_t)) + align_up(sizeof(uint32_t) * 4);
}

hipError_t launch_preprocess(const GaussPtrs& g, const ws_camera* d_cams, int32_t n_views, const KOpts& o,
                             ws_splat* splats, uint32_t* tiles_touched, uint64_t* keys, uint32_t* values,
                             int64_t capacity, int64_t* d_num_pairs, int32_t* d_status, void* ws,
                             hipStream_t stream) {
    PreprocessWs pw = carve(ws, g.n, n_views);
    const int64_t total = g.n * n_views;
    const uint32_t gx = uint32_t(std::max<int64_t>((g.n + kPreThreads - 1) / kPreThreads, 1));
    timing_begin(WS_KERNEL_PREPROCESS, stream);
    switch (o.sh_degree) {
        case 0: hipLaunchKernelGGL(k_preprocess<0>, dim3(gx, n_views), dim3(kPreThreads), 0, stream, g, d_cams, o,
                                   splats, tiles_touched, pw); break;
        case 1: hipLaunchKernelGGL(k_preprocess<1>, dim3(gx, n_views), dim3(kPreThreads), 0, stream, g, d_cams, o,
                                   splats, tiles_touched, pw); break;
        case 2: hipLaunchKernelGGL(k_preprocess<2>, dim3(gx, n_views), dim3(kPreThreads), 0, stream, g, d_cams, o,
                                   splats, tiles_touched, pw); break;
        default: hipLaunchKernelGGL(k_preprocess<3>, dim3(gx, n_views), dim3(kPreThreads), 0, stream, g, d_cams, o,
                                    splats, tiles_touched, pw); break;
    }
    timing_end(WS_KERNEL_PREPROCESS, stream);
    EmitArgs a;
    a.tiles_touched = tiles_touched;
    a.splats = splats;
    a.cams = d_cams;
    a.n_views = n_views;
    a.n = std::max<int64_t>(g.n, 1);
    a.total = total;
    a.tile_w = o.tile_w;
    a.tile_h = o.tile_h;
    a.keys = keys;
    a.values = values;
    a.capacity = capacity;
    a.d_num_pairs = d_num_pairs;
    a.d_status = d_status;
    const uint32_t blocks = uint32_t(std::max<int64_t>(pw.n_blocks, 1));
    a.n_launched = blocks;  // with no Gaussians one block still reports M = 0
    timing_begin(WS_KERNEL_SCAN_EMIT, stream);
    hipLaunchKernelGGL(k_scan_emit, dim3(blocks), dim3(kScanThreads), 0, stream, a, pw);
    timing_end(WS_KERNEL_SCAN_EMIT, stream);
    return hipGetLastError();
}

}  // namespace ws
