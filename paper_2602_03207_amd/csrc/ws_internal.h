// Internal declarations of the websplat HIP library (gfx950, wave64).
// Device helpers shared by the kernels and the host-side launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdlib>

#include "../../include/websplat.h"

namespace ws {

constexpr int kWave = 64;

// ------------------------------------------------------------ wave helpers

// Number of set bits of `mask` below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// DPP move of a 32-bit value by the control word CTRL (row_shr, row_bcast,
// wave_shr, ...), rows outside ROW_MASK and lanes without a source read 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ uint32_t dpp_move(uint32_t v) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, ROW_MASK, 0xf, false));
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ uint64_t dpp_move(uint64_t v) {
    return uint64_t(dpp_move<CTRL, ROW_MASK>(uint32_t(v))) | (uint64_t(dpp_move<CTRL, ROW_MASK>(uint32_t(v >> 32))) << 32);
}

// The value of lane 63 (uniform).
__device__ __forceinline__ uint32_t last_lane(uint32_t v) {
    return uint32_t(__builtin_amdgcn_readlane(int(v), kWave - 1));
}
__device__ __forceinline__ uint64_t last_lane(uint64_t v) {
    return uint64_t(last_lane(uint32_t(v))) | (uint64_t(last_lane(uint32_t(v >> 32))) << 32);
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_move(float v) {
    return __builtin_bit_cast(float, dpp_move<CTRL, ROW_MASK>(__builtin_bit_cast(uint32_t, v)));
}
__device__ __forceinline__ float last_lane(float v) {
    return __builtin_bit_cast(float, last_lane(__builtin_bit_cast(uint32_t, v)));
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_move(double v) {
    return __builtin_bit_cast(double, dpp_move<CTRL, ROW_MASK>(__builtin_bit_cast(uint64_t, v)));
}
__device__ __forceinline__ double last_lane(double v) {
    return __builtin_bit_cast(double, last_lane(__builtin_bit_cast(uint64_t, v)));
}

// Inclusive prefix sum across the 64 lanes of a wave (32- or 64-bit):
// shifts by 1, 2, 4 and 8 within each row of 16 lanes, then the broadcast of
// lane 15 into rows 1 and 3 and of lane 31 into rows 2 and 3 -- DPP operands
// of ordinary adds, no LDS round trips.
template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    v += dpp_move<0x111>(v);  // row_shr 1
    v += dpp_move<0x112>(v);  // row_shr 2
    v += dpp_move<0x114>(v);  // row_shr 4
    v += dpp_move<0x118>(v);  // row_shr 8
    v += dpp_move<0x142, 0xa>(v);  // row_bcast 15
    v += dpp_move<0x143, 0xc>(v);  // row_bcast 31
    return v;
}


// Sum over the 64 lanes of a wave, as a uniform value (the last lane of the
// DPP prefix sum).
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
    return last_lane(wave_inclusive_scan(v));
}

// Workgroups of a 1-D grid are dealt to the 8 XCDs round-robin by blockIdx.
// This maps block b < count to a work item so that each XCD receives one
// contiguous range of items (a bijection on [0, count)): neighbouring items
// then share that XCD's L2, and lines they write in part are merged there.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t count) {
    const uint32_t x = b % kXcds, q = count / kXcds, r = count % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

// Exclusive prefix sum over a workgroup of NT threads (NT a multiple of 64).
// `scratch` holds NT/64 + 1 values; returns the exclusive prefix and the total.
template <int NT, class T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* scratch, T* total) {
    constexpr int NW = NT / kWave;
    const int wave = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    T inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) scratch[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int w = 0; w < NW; ++w) {
            T c = scratch[w];
            scratch[w] = run;
            run += c;
        }
        scratch[NW] = run;
    }
    __syncthreads();
    T res = scratch[wave] + inc - v;
    *total = scratch[NW];
    __syncthreads();
    return res;
}

// ------------------------------------------------ device-scope atomics

__device__ __forceinline__ uint64_t load_agent(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_agent(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Widest digit of a radix sort pass (bits).
constexpr int kMaxRadixBits = 10;

// Bounded waits: a look-back that has not seen its predecessor after this
// many polls gives up and reports WS_ERR_SPIN_LIMIT instead of hanging.
constexpr uint32_t kSpinLimit = 1u << 22;

// Synchronisation words (look-back flags, global histograms) must be
// zero when the kernel that uses them starts.  Instead of a clearing launch of
// its own (a few microseconds each, most of it the dependency between
// back-to-back launches), an earlier kernel of the same stream that does not
// use the words zeroes them with its spare threads.
struct ClearList {
    static constexpr int kMax = 4;
    uint32_t* ptr[kMax];
    int64_t words[kMax];
    int count = 0;
    void add(void* p, int64_t w) {
        if (!p || w <= 0) return;
        if (count == kMax) std::abort();  // a fixed number of regions per launch: a programming error
        ptr[count] = static_cast<uint32_t*>(p);
        words[count++] = w;
    }
};

// Called by every thread of the clearing kernel: `gid` is its index in the
// grid, `threads` the grid's thread count.
__device__ __forceinline__ void clear_words(const ClearList& c, int64_t gid, int64_t threads) {
    for (int r = 0; r < c.count; ++r)
        for (int64_t i = gid; i < c.words[r]; i += threads) c.ptr[r][i] = 0u;
}

// ------------------------------------------------------- shared data

struct GaussPtrs {
    const float* means;
    const float* log_scales;
    const float* quats;
    const float* logits;
    const float* sh;
    int64_t n;
};

struct GradPtrs {
    float* means;
    float* log_scales;
    float* quats;
    float* logits;
    float* sh;
};

// Options as the kernels see them.
struct KOpts {
    int32_t tile_w, tile_h, sh_degree;
    uint32_t flags;
    float near_z, lowpass, clamp_fov, alpha_min, alpha_max, t_min;
    float bg[3];
    int32_t bin_x, bin_y;  // tiles per key cell (1, 2, 4 or 8)
    // Bins only: the bit of the key's cell word (the high word of a 64-bit
    // key, a 32-bit key itself) where the mask of the bin's tiles that the
    // splat covers starts (= the bits of the cell id); -1 without a mask.
    int32_t mask_shift;
    // pixel size of the cells that pair keys name: a tile, or a bin of tiles
    __host__ __device__ int32_t cell_w() const { return tile_w * bin_x; }
    __host__ __device__ int32_t cell_h() const { return tile_h * bin_y; }
    // the cell id bits of a key's cell word
    __host__ __device__ uint32_t cell_mask() const {
        return mask_shift < 0 ? 0xffffffffu : (1u << mask_shift) - 1u;
    }
};

inline KOpts to_kopts(const ws_options& o) {
    KOpts k;
    k.tile_w = o.tile_w; k.tile_h = o.tile_h; k.sh_degree = o.sh_degree; k.flags = o.flags;
    k.bin_x = o.bin_x > 1 ? o.bin_x : 1;
    k.bin_y = o.bin_y > 1 ? o.bin_y : 1;
    k.mask_shift = -1;  // set by the caller that knows the cameras (bins only)
    k.near_z = o.near_z; k.lowpass = o.lowpass; k.clamp_fov = o.clamp_fov;
    k.alpha_min = o.alpha_min; k.alpha_max = o.alpha_max; k.t_min = o.t_min;
    k.bg[0] = o.bg[0]; k.bg[1] = o.bg[1]; k.bg[2] = o.bg[2];
    return k;
}

__host__ __device__ inline int32_t ceil_div(int32_t a, int32_t b) { return (a + b - 1) / b; }

// Tile id offset and image float offset of view v, from the device cameras
// (n_views is small; a linear pass is cheaper than a table).
__device__ __forceinline__ void view_offsets(const ws_camera* cams, int32_t v, int32_t tw, int32_t th,
                                             int64_t* tile_off, int64_t* img_off) {
    int64_t t = 0, f = 0;
    for (int32_t u = 0; u < v; ++u) {
        const int32_t W = cams[u].width, H = cams[u].height;
        t += int64_t(ceil_div(W, tw)) * ceil_div(H, th);
        f += 3ll * W * H;
    }
    *tile_off = t;
    *img_off = f;
}

// ---------------------------------------------------- launchers (host)

// preprocess.hip
// keys: uint64_t (cell << 32 | depth bits), or uint32_t cell ids with WS_FLAG_KEYS32
hipError_t launch_preprocess(const GaussPtrs& g, const ws_camera* d_cams, int32_t n_views, const KOpts& o,
                             ws_splat* splats, uint32_t* tiles_touched, void* keys, uint32_t* values,
                             int64_t capacity, int64_t* d_num_pairs, int32_t* d_status, void* ws,
                             hipStream_t stream);
size_t preprocess_workspace(int64_t n, int32_t n_views, int64_t capacity, uint32_t flags);

// sort.hip
// `timed`: report the launches to the benchmark timing hooks (false for sorts
// made inside another stage, which that stage's timing already covers).
// `sparse`: the device count is expected to be far below the capacity; the
// sort then always takes the small-tile look-back schedule, whose cost follows
// the live count (workgroups past it leave at once) rather than the capacity.
// `precleared`: an earlier kernel of the stream zeroed the words that
// sort_sync_words lists, so the sort launches no clearing kernel.
// The two overloads sort 64-bit and 32-bit keys; key_bytes below is 8 or 4.
// `hist_ready`: an earlier kernel filled the histograms and cleared the
// look-back words listed by sort_hist_words (look-back schedule only).
hipError_t launch_sort(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout, int64_t n,
                       const int64_t* d_n, const int32_t* d_status, int32_t begin_bit, int32_t end_bit,
                       int32_t radix_bits, void* ws, hipStream_t stream, bool timed = true, bool sparse = false,
                       bool precleared = false, bool hist_ready = false);
hipError_t launch_sort(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, int64_t n,
                       const int64_t* d_n, const int32_t* d_status, int32_t begin_bit, int32_t end_bit,
                       int32_t radix_bits, void* ws, hipStream_t stream, bool timed = true, bool sparse = false,
                       bool precleared = false, bool hist_ready = false);
size_t sort_workspace(int64_t capacity, int32_t begin_bit, int32_t end_bit, int32_t radix_bits, bool sparse = false,
                      int key_bytes = 8);
// Adds to `c` the words of a sort with these arguments that must be zero when
// it starts (none for the wait-free schedule, whose passes clear their own).
void sort_sync_words(void* ws, int64_t capacity, int32_t begin_bit, int32_t end_bit, int32_t radix_bits, bool sparse,
                     int key_bytes, ClearList* c);
// The digit histograms and look-back words of a look-back (sparse or small)
// sort with these arguments, for a kernel that produces the sort's input and
// fills them on the way (launch_sort with hist_ready then skips its histogram
// kernel): hist [passes][radix] (zero when the producer starts, then the digit
// counts of every pass), status [passes][max_tiles][radix] (the words of every
// tile holding input zeroed by the producer), tiles of `tile` pairs.
struct SortHistWords {
    uint32_t* hist;
    uint32_t* status;
    int64_t max_tiles;
    int passes, radix, r, tile;
};
SortHistWords sort_hist_words(void* ws, int64_t capacity, int32_t begin_bit, int32_t end_bit, int32_t radix_bits,
                              bool sparse, int key_bytes);

// render.hip
hipError_t launch_render(const ws_splat* splats, int64_t n, const ws_camera* d_cams, int32_t n_views,
                         int64_t total_tiles, const KOpts& o, const void* keys, const uint32_t* values,
                         int64_t capacity, const int64_t* d_num_pairs, const int32_t* d_status,
                         uint32_t* tile_ranges, float* images, void* ws, hipStream_t stream);
size_t render_workspace(int64_t total_tiles, const KOpts& o);
size_t expand_workspace(int64_t total_bins);
hipError_t launch_expand(const ws_splat* splats, int64_t n, const ws_camera* d_cams, int32_t n_views,
                         int64_t total_bins, const KOpts& o, const void* keys, const uint32_t* values,
                         int64_t capacity, const int64_t* d_num_pairs, const int32_t* d_status,
                         uint32_t* tile_values, uint32_t* tile_ranges, void* ws, hipStream_t stream);

// backward.hip
// The L1 loss formed inside the compositing adjoint (ws_render_backward_l1).
struct L1Loss {
    const float* targets;
    int64_t total;  // elements the mean is taken over
    float* d_loss;
};
hipError_t launch_render_backward(const GaussPtrs& g, const ws_camera* d_cams, int32_t n_views,
                                  int64_t total_tiles, const KOpts& o, const ws_splat* splats,
                                  const uint32_t* tiles_touched, const uint32_t* values, const uint32_t* tile_ranges, const float* images,
                                  const float* dL_dimages, const int32_t* d_status, const GradPtrs& grads, void* ws,
                                  hipStream_t stream, const L1Loss* l1 = nullptr);
size_t render_backward_l1_workspace(int64_t n, int32_t n_views, int64_t total_tiles);
// *loss = sum of partial[0..nb) / total in a fixed order; nothing when *d_status != 0 (d_status may be null).
void launch_l1_final(const double* partial, int64_t nb, int64_t total, const int32_t* d_status, float* loss,
                     hipStream_t stream);
size_t render_backward_workspace(int64_t n, int32_t n_views);

// loss.hip
hipError_t launch_l1_loss(const float* images, const float* targets, int64_t n, int64_t total, float* dL,
                          float* d_loss, void* ws, hipStream_t stream);
size_t l1_loss_workspace(int64_t n);

// Benchmark timing hooks (defined in api.hip): no-ops unless ws_timing_start
// selected this kernel.
void timing_begin(int kernel, hipStream_t stream);
void timing_end(int kernel, hipStream_t stream);

// noalloc.hip: the allocation-free sort's scratch, a file-scope device array
// of kStaticScratchBytes per GPU.  static_scratch() returns its device address
// on the current device (looked up once per device).
constexpr int64_t kStaticScratchMaxPairs = int64_t(1) << 20;
constexpr size_t kStaticScratchBytes = size_t(24) << 20;
hipError_t static_scratch(void** ptr);

// Round a byte count up to the workspace alignment.
inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

}  // namespace ws
