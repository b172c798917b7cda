// C ABI of libwebsplat: argument validation, workspace sizing, error
// reporting and HIP-graph helpers.  Every check here runs on the host before
// any work is enqueued, so a rejected call leaves the stream untouched.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "ws_internal.h"

namespace {

thread_local std::string g_last_error;

ws_status fail(ws_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

ws_status hip_status(hipError_t e, const char* where) {
    if (e == hipSuccess) return WS_OK;
    return fail(WS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

constexpr int32_t kMaxViews = 4096;
constexpr int64_t kMaxGaussians = (int64_t(1) << 31) - 1;
constexpr int64_t kMaxSortN = (int64_t(1) << 30) - 1;

bool finite_pos(float x) { return std::isfinite(x) && x > 0.f; }

ws_status check_options(const ws_options* o) {
    if (!o) return fail(WS_ERR_INVALID_ARGUMENT, "options is NULL");
    const bool tile_ok = (o->tile_w == 16 && o->tile_h == 16) || (o->tile_w == 8 && o->tile_h == 8) ||
                         (o->tile_w == 16 && o->tile_h == 8) || (o->tile_w == 32 && o->tile_h == 16);
    if (!tile_ok) return fail(WS_ERR_UNSUPPORTED, "tile size %dx%d not supported (16x16, 8x8, 16x8, 32x16)",
                              o->tile_w, o->tile_h);
    if (o->sh_degree < 0 || o->sh_degree > 3)
        return fail(WS_ERR_UNSUPPORTED, "sh_degree %d not supported (0..3)", o->sh_degree);
    if (o->radix_bits < 0 || o->radix_bits > ws::kMaxRadixBits)
        return fail(WS_ERR_INVALID_ARGUMENT, "radix_bits %d out of range (0..%d)", o->radix_bits, ws::kMaxRadixBits);
    for (const int32_t b : {o->bin_x, o->bin_y})
        if (b != 0 && b != 1 && b != 2 && b != 4 && b != 8)
            return fail(WS_ERR_INVALID_ARGUMENT, "bin_x / bin_y must be 1, 2, 4 or 8 (0 reads as 1), got %d", b);
    if (o->flags & ~(WS_FLAG_FIXED_3SIGMA | WS_FLAG_NO_VIEWPORT_CULL | WS_FLAG_ORDERED_RENDER | WS_FLAG_DEPTH_FIRST |
                     WS_FLAG_KEYS32 | WS_FLAG_ACCUMULATE_GRADS | WS_FLAG_PACKED))
        return fail(WS_ERR_INVALID_ARGUMENT, "unknown flag bits 0x%x", o->flags);
    if ((o->flags & WS_FLAG_KEYS32) && !(o->flags & WS_FLAG_DEPTH_FIRST))
        return fail(WS_ERR_INVALID_ARGUMENT, "WS_FLAG_KEYS32 needs WS_FLAG_DEPTH_FIRST (the keys carry no depth)");
    if (!finite_pos(o->near_z)) return fail(WS_ERR_INVALID_ARGUMENT, "near_z must be finite and > 0");
    if (!(std::isfinite(o->lowpass) && o->lowpass >= 0.f))
        return fail(WS_ERR_INVALID_ARGUMENT, "lowpass must be finite and >= 0");
    if (!finite_pos(o->clamp_fov)) return fail(WS_ERR_INVALID_ARGUMENT, "clamp_fov must be finite and > 0");
    if (!(o->alpha_min > 0.f && o->alpha_min < 1.f))
        return fail(WS_ERR_INVALID_ARGUMENT, "alpha_min must lie in (0, 1)");
    if (!(o->alpha_max >= o->alpha_min && o->alpha_max < 1.f))
        return fail(WS_ERR_INVALID_ARGUMENT, "alpha_max must lie in [alpha_min, 1)");
    if (!(o->t_min > 0.f && o->t_min < 1.f)) return fail(WS_ERR_INVALID_ARGUMENT, "t_min must lie in (0, 1)");
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(o->bg[c])) return fail(WS_ERR_INVALID_ARGUMENT, "bg must be finite");
    return WS_OK;
}

ws_status check_cameras(const ws_camera* cams, const ws_camera* d_cams, int32_t n_views) {
    if (n_views < 1 || n_views > kMaxViews)
        return fail(WS_ERR_INVALID_ARGUMENT, "n_views %d out of range (1..%d)", n_views, kMaxViews);
    if (!cams) return fail(WS_ERR_INVALID_ARGUMENT, "cams (host) is NULL");
    if (!d_cams) return fail(WS_ERR_INVALID_ARGUMENT, "d_cams (device) is NULL");
    for (int32_t v = 0; v < n_views; ++v) {
        const ws_camera& c = cams[v];
        if (c.width < 1 || c.width > 32767 || c.height < 1 || c.height > 32767)
            return fail(WS_ERR_INVALID_ARGUMENT, "camera %d: size %dx%d out of range", v, c.width, c.height);
        if (!finite_pos(c.fx) || !finite_pos(c.fy) || !std::isfinite(c.cx) || !std::isfinite(c.cy))
            return fail(WS_ERR_INVALID_ARGUMENT, "camera %d: intrinsics must be finite, fx and fy > 0", v);
        for (int k = 0; k < 9; ++k)
            if (!std::isfinite(c.R[k])) return fail(WS_ERR_INVALID_ARGUMENT, "camera %d: R not finite", v);
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(c.t[k]) || !std::isfinite(c.C[k]))
                return fail(WS_ERR_INVALID_ARGUMENT, "camera %d: t or C not finite", v);
    }
    return WS_OK;
}

ws_status check_gaussians(const ws_gaussians* g) {
    if (!g) return fail(WS_ERR_INVALID_ARGUMENT, "gaussians is NULL");
    if (g->n < 0 || g->n > kMaxGaussians)
        return fail(WS_ERR_INVALID_ARGUMENT, "n = %lld out of range (0..2^31-1)", (long long)g->n);
    if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh))
        return fail(WS_ERR_INVALID_ARGUMENT, "a Gaussian parameter array is NULL");
    return WS_OK;
}

ws_status check_ws(const void* ws, size_t ws_bytes, size_t need) {
    if (ws_bytes < need)
        return fail(WS_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (need > 0 && !ws) return fail(WS_ERR_INVALID_ARGUMENT, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return fail(WS_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
    return WS_OK;
}

int64_t total_tiles_of(const ws_camera* cams, int32_t n_views, int32_t tw, int32_t th) {
    int64_t t = 0;
    for (int32_t v = 0; v < n_views; ++v) t += int64_t(ws::ceil_div(cams[v].width, tw)) * ws::ceil_div(cams[v].height, th);
    return t;
}

// Key cells of the views: tiles, or bins of bin_x x bin_y tiles.
int64_t total_bins_of(const ws_camera* cams, int32_t n_views, const ws_options* o) {
    const ws::KOpts k = ws::to_kopts(*o);
    return total_tiles_of(cams, n_views, k.cell_w(), k.cell_h());
}

bool binned(const ws_options* o) { return o->bin_x > 1 || o->bin_y > 1; }

// Kernel options with the position of the bins' coverage mask in the key's
// cell word: above the ceil(log2(total bins)) bits of the bin id (at least 1),
// when those bits and one bit per tile of a bin fit in 32.
ws::KOpts kopts_for(const ws_options* o, const ws_camera* cams, int32_t n_views) {
    ws::KOpts k = ws::to_kopts(*o);
    if (!binned(o)) return k;
    const int64_t bins = total_bins_of(cams, n_views, o);
    int32_t bits = 1;
    while ((int64_t(1) << bits) < bins) ++bits;
    if (bits + k.bin_x * k.bin_y <= 32) k.mask_shift = bits;
    return k;
}

ws::GaussPtrs gauss_ptrs(const ws_gaussians* g) {
    ws::GaussPtrs p;
    p.means = g->means;
    p.log_scales = g->log_scales;
    p.quats = g->quats;
    p.logits = g->opacity_logits;
    p.sh = g->sh;
    p.n = g->n;
    return p;
}

bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bn && y < x + an;
}

struct Timing {
    int kernel = -1;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    size_t used = 0;
    bool open = false;
};
Timing g_timing;
constexpr size_t kTimingSlots = 4096;

}  // namespace

namespace ws {

void timing_begin(int kernel, hipStream_t stream) {
    if (g_timing.kernel != kernel || g_timing.used >= g_timing.pool.size()) return;
    (void)hipEventRecord(g_timing.pool[g_timing.used].first, stream);
    g_timing.open = true;
}

void timing_end(int kernel, hipStream_t stream) {
    if (g_timing.kernel != kernel || !g_timing.open) return;
    (void)hipEventRecord(g_timing.pool[g_timing.used].second, stream);
    g_timing.open = false;
    ++g_timing.used;
}

}  // namespace ws

extern "C" {

ws_status ws_timing_start(int32_t kernel) {
    if (kernel < WS_KERNEL_PREPROCESS || kernel > WS_KERNEL_PREPROCESS_BWD)
        return fail(WS_ERR_INVALID_ARGUMENT, "unknown kernel id %d", kernel);
    while (g_timing.pool.size() < kTimingSlots) {
        hipEvent_t a = nullptr, b = nullptr;
        ws_status s = hip_status(hipEventCreate(&a), "hipEventCreate");
        if (s != WS_OK) return s;
        s = hip_status(hipEventCreate(&b), "hipEventCreate");
        if (s != WS_OK) return s;
        g_timing.pool.emplace_back(a, b);
    }
    g_timing.kernel = kernel;
    g_timing.used = 0;
    g_timing.open = false;
    return WS_OK;
}

ws_status ws_timing_stop(double* total_ms, int64_t* launches) {
    if (!total_ms || !launches) return fail(WS_ERR_INVALID_ARGUMENT, "total_ms / launches is NULL");
    double sum = 0.0;
    for (size_t k = 0; k < g_timing.used; ++k) {
        ws_status s = hip_status(hipEventSynchronize(g_timing.pool[k].second), "hipEventSynchronize");
        if (s != WS_OK) return s;
        float ms = 0.f;
        s = hip_status(hipEventElapsedTime(&ms, g_timing.pool[k].first, g_timing.pool[k].second),
                       "hipEventElapsedTime");
        if (s != WS_OK) return s;
        sum += ms;
    }
    *total_ms = sum;
    *launches = int64_t(g_timing.used);
    g_timing.kernel = -1;
    g_timing.used = 0;
    return WS_OK;
}

int32_t ws_version(void) { return 10100; }

const char* ws_last_error(void) { return g_last_error.c_str(); }

const char* ws_status_string(int32_t s) {
    switch (s) {
        case WS_OK: return "ok";
        case WS_ERR_INVALID_ARGUMENT: return "invalid argument";
        case WS_ERR_UNSUPPORTED: return "unsupported";
        case WS_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case WS_ERR_HIP: return "HIP error";
        case WS_ERR_CAPACITY: return "pair capacity exceeded";
        case WS_ERR_SPIN_LIMIT: return "bounded wait expired";
        default: return "unknown status";
    }
}

size_t ws_preprocess_workspace_size(int64_t n, int32_t n_views, int64_t capacity, uint32_t flags) {
    if (n < 0 || n_views < 1) return 0;
    return ws::preprocess_workspace(n, n_views, capacity < 0 ? 0 : capacity, flags);
}

size_t ws_sort_workspace_size(int64_t capacity, int32_t begin_bit, int32_t end_bit, int32_t radix_bits) {
    if (capacity < 0 || begin_bit < 0 || end_bit > 64 || begin_bit >= end_bit || radix_bits < 0 ||
        radix_bits > ws::kMaxRadixBits)
        return 0;
    return ws::sort_workspace(capacity, begin_bit, end_bit, radix_bits, false, 8);
}

size_t ws_sort32_workspace_size(int64_t capacity, int32_t begin_bit, int32_t end_bit, int32_t radix_bits) {
    if (capacity < 0 || begin_bit < 0 || end_bit > 32 || begin_bit >= end_bit || radix_bits < 0 ||
        radix_bits > ws::kMaxRadixBits)
        return 0;
    return ws::sort_workspace(capacity, begin_bit, end_bit, radix_bits, false, 4);
}

int64_t ws_total_tiles(const ws_camera* cams, int32_t n_views, const ws_options* opt) {
    if (!cams || !opt || n_views < 1 || opt->tile_w < 1 || opt->tile_h < 1) return -1;
    return total_tiles_of(cams, n_views, opt->tile_w, opt->tile_h);
}

int64_t ws_total_bins(const ws_camera* cams, int32_t n_views, const ws_options* opt) {
    if (!cams || !opt || n_views < 1 || opt->tile_w < 1 || opt->tile_h < 1 || opt->bin_x < 0 || opt->bin_y < 0)
        return -1;
    return total_bins_of(cams, n_views, opt);
}

size_t ws_expand_bins_workspace_size(const ws_camera* cams, int32_t n_views, const ws_options* opt) {
    if (ws_total_bins(cams, n_views, opt) < 0) return 0;
    return ws::expand_workspace(total_bins_of(cams, n_views, opt));
}

int64_t ws_total_image_floats(const ws_camera* cams, int32_t n_views) {
    if (!cams || n_views < 1) return -1;
    int64_t f = 0;
    for (int32_t v = 0; v < n_views; ++v) f += 3ll * cams[v].width * cams[v].height;
    return f;
}

size_t ws_render_workspace_size(const ws_camera* cams, int32_t n_views, const ws_options* opt) {
    if (!cams || !opt || n_views < 1 || opt->tile_w < 1 || opt->tile_h < 1) return 0;
    return ws::render_workspace(total_tiles_of(cams, n_views, opt->tile_w, opt->tile_h), ws::to_kopts(*opt));
}

size_t ws_render_backward_workspace_size(int64_t n, int32_t n_views) {
    if (n < 0 || n_views < 1) return 0;
    return ws::render_backward_workspace(n, n_views);
}

size_t ws_render_backward_l1_workspace_size(int64_t n, const ws_camera* cams, int32_t n_views,
                                           const ws_options* opt) {
    if (n < 0 || n_views < 1 || !cams || !opt) return 0;
    return ws::render_backward_l1_workspace(n, n_views, total_tiles_of(cams, n_views, opt->tile_w, opt->tile_h));
}

size_t ws_l1_loss_workspace_size(int64_t n) {
    if (n < 0) return 0;
    return ws::l1_loss_workspace(n);
}

ws_status ws_preprocess(const ws_gaussians* g, const ws_camera* cams, const ws_camera* d_cams, int32_t n_views,
                        const ws_options* opt, ws_splat* splats, uint32_t* tiles_touched, void* keys,
                        uint32_t* values, int64_t capacity, int64_t* d_num_pairs, int32_t* d_status, void* ws,
                        size_t ws_bytes, void* stream) {
    ws_status s;
    if ((s = check_gaussians(g)) != WS_OK) return s;
    if ((s = check_cameras(cams, d_cams, n_views)) != WS_OK) return s;
    if ((s = check_options(opt)) != WS_OK) return s;
    if (g->n * int64_t(n_views) > kMaxGaussians)
        return fail(WS_ERR_INVALID_ARGUMENT, "n * n_views must be < 2^31");
    if (g->n > 0 && (!splats || !tiles_touched))
        return fail(WS_ERR_INVALID_ARGUMENT, "splats / tiles_touched is NULL");
    if (capacity < 0) return fail(WS_ERR_INVALID_ARGUMENT, "capacity < 0");
    if (capacity > 0 && (!keys || !values)) return fail(WS_ERR_INVALID_ARGUMENT, "keys / values is NULL");
    if (!d_num_pairs || !d_status) return fail(WS_ERR_INVALID_ARGUMENT, "d_num_pairs / d_status is NULL");
    if (total_bins_of(cams, n_views, opt) > (int64_t(1) << 32))
        return fail(WS_ERR_UNSUPPORTED, "more than 2^32 tiles (bins)");
    if ((s = check_ws(ws, ws_bytes, ws::preprocess_workspace(g->n, n_views, capacity, opt->flags))) != WS_OK) return s;
    if (reinterpret_cast<uintptr_t>(splats) % 16 != 0)
        return fail(WS_ERR_INVALID_ARGUMENT, "splats must be 16-byte aligned");
    const hipError_t e = ws::launch_preprocess(gauss_ptrs(g), d_cams, n_views, kopts_for(opt, cams, n_views), splats,
                                               tiles_touched, keys, values, capacity, d_num_pairs, d_status, ws,
                                               static_cast<hipStream_t>(stream));
    return hip_status(e, "ws_preprocess launch");
}

extern "C++" {
namespace {

template <typename K>
ws_status sort_checked(const char* name, const K* keys_in, const uint32_t* values_in, K* keys_out,
                       uint32_t* values_out, int64_t n, const int64_t* d_n, const int32_t* d_status, int32_t begin_bit,
                       int32_t end_bit, int32_t radix_bits, void* ws, size_t ws_bytes, void* stream) {
    constexpr int kBits = int(sizeof(K)) * 8;
    if (n < 0 || n > kMaxSortN)
        return fail(WS_ERR_INVALID_ARGUMENT, "%s: n = %lld out of range (0..2^30-1)", name, (long long)n);
    if (begin_bit < 0 || end_bit > kBits || begin_bit >= end_bit)
        return fail(WS_ERR_INVALID_ARGUMENT, "%s: need 0 <= begin_bit < end_bit <= %d (got %d, %d)", name, kBits,
                    begin_bit, end_bit);
    if (radix_bits < 0 || radix_bits > ws::kMaxRadixBits)
        return fail(WS_ERR_INVALID_ARGUMENT, "%s: radix_bits %d out of range (0..%d)", name, radix_bits,
                    ws::kMaxRadixBits);
    if (n == 0) return WS_OK;
    if (!keys_in || !values_in || !keys_out || !values_out)
        return fail(WS_ERR_INVALID_ARGUMENT, "%s: a key/value pointer is NULL", name);
    if (overlaps(keys_in, size_t(n) * sizeof(K), keys_out, size_t(n) * sizeof(K)) ||
        overlaps(values_in, size_t(n) * 4, values_out, size_t(n) * 4))
        return fail(WS_ERR_INVALID_ARGUMENT, "%s: output buffers must not overlap the inputs", name);
    ws_status s;
    if ((s = check_ws(ws, ws_bytes, ws::sort_workspace(n, begin_bit, end_bit, radix_bits, false, int(sizeof(K))))) !=
        WS_OK)
        return s;
    const hipError_t e = ws::launch_sort(keys_in, values_in, keys_out, values_out, n, d_n, d_status, begin_bit,
                                         end_bit, radix_bits, ws, static_cast<hipStream_t>(stream));
    return hip_status(e, name);
}

}  // namespace
}  // extern "C++"

ws_status ws_sort(const uint64_t* keys_in, const uint32_t* values_in, uint64_t* keys_out, uint32_t* values_out,
                  int64_t n, const int64_t* d_n, const int32_t* d_status, int32_t begin_bit, int32_t end_bit,
                  int32_t radix_bits, void* ws, size_t ws_bytes, void* stream) {
    return sort_checked("ws_sort", keys_in, values_in, keys_out, values_out, n, d_n, d_status, begin_bit, end_bit,
                        radix_bits, ws, ws_bytes, stream);
}

ws_status ws_sort32(const uint32_t* keys_in, const uint32_t* values_in, uint32_t* keys_out, uint32_t* values_out,
                    int64_t n, const int64_t* d_n, const int32_t* d_status, int32_t begin_bit, int32_t end_bit,
                    int32_t radix_bits, void* ws, size_t ws_bytes, void* stream) {
    return sort_checked("ws_sort32", keys_in, values_in, keys_out, values_out, n, d_n, d_status, begin_bit, end_bit,
                        radix_bits, ws, ws_bytes, stream);
}

ws_status ws_sort_noalloc(const uint64_t* keys_in, const uint32_t* values_in, uint64_t* keys_out,
                          uint32_t* values_out, int64_t n, const int64_t* d_n, const int32_t* d_status,
                          int32_t begin_bit, int32_t end_bit, int32_t radix_bits, void* stream) {
    if (n < 0 || n > ws::kStaticScratchMaxPairs)
        return fail(WS_ERR_INVALID_ARGUMENT,
                    "ws_sort_noalloc: n = %lld exceeds the static scratch's maximum of %lld pairs (use ws_sort)",
                    (long long)n, (long long)ws::kStaticScratchMaxPairs);
    if (n == 0) return WS_OK;
    void* scratch = nullptr;
    const hipError_t e = ws::static_scratch(&scratch);
    if (e != hipSuccess) return hip_status(e, "ws_sort_noalloc: static scratch");
    // the same validation and kernels as ws_sort, with the static scratch as the workspace
    return sort_checked("ws_sort_noalloc", keys_in, values_in, keys_out, values_out, n, d_n, d_status, begin_bit,
                        end_bit, radix_bits, scratch, ws::kStaticScratchBytes, stream);
}

ws_status ws_render(const ws_splat* splats, int64_t n, const ws_camera* cams, const ws_camera* d_cams,
                    int32_t n_views, const ws_options* opt, const void* keys, const uint32_t* values,
                    int64_t capacity, const int64_t* d_num_pairs, const int32_t* d_status, uint32_t* tile_ranges,
                    float* images, void* ws, size_t ws_bytes, void* stream) {
    ws_status s;
    if (n < 0 || n > kMaxGaussians) return fail(WS_ERR_INVALID_ARGUMENT, "n out of range");
    if ((s = check_cameras(cams, d_cams, n_views)) != WS_OK) return s;
    if ((s = check_options(opt)) != WS_OK) return s;
    if (capacity < 0 || capacity > (int64_t(1) << 32) - 1) return fail(WS_ERR_INVALID_ARGUMENT, "capacity out of range");
    if (capacity > 0 && !values) return fail(WS_ERR_INVALID_ARGUMENT, "values is NULL");
    if (binned(opt) && keys)
        return fail(WS_ERR_INVALID_ARGUMENT, "with bins larger than one tile, pass keys = NULL and the lists and "
                                             "ranges of ws_expand_bins");
    if (n > 0 && !splats) return fail(WS_ERR_INVALID_ARGUMENT, "splats is NULL");
    if (!d_status || !tile_ranges || !images)
        return fail(WS_ERR_INVALID_ARGUMENT, "d_status / tile_ranges / images is NULL");
    if (keys && !d_num_pairs) return fail(WS_ERR_INVALID_ARGUMENT, "d_num_pairs is NULL");
    const int64_t tiles = total_tiles_of(cams, n_views, opt->tile_w, opt->tile_h);
    if (tiles > (int64_t(1) << 31)) return fail(WS_ERR_UNSUPPORTED, "more than 2^31 tiles");
    const ws::KOpts ko = kopts_for(opt, cams, n_views);
    if ((s = check_ws(ws, ws_bytes, ws::render_workspace(tiles, ko))) != WS_OK) return s;
    const hipError_t e = ws::launch_render(splats, n, d_cams, n_views, tiles, ko, keys, values, capacity, d_num_pairs,
                                           d_status, tile_ranges, images, ws, static_cast<hipStream_t>(stream));
    return hip_status(e, "ws_render launch");
}

ws_status ws_expand_bins(const ws_splat* splats, int64_t n, const ws_camera* cams, const ws_camera* d_cams,
                         int32_t n_views, const ws_options* opt, const void* keys, const uint32_t* values,
                         int64_t capacity, const int64_t* d_num_pairs, const int32_t* d_status,
                         uint32_t* tile_values, int64_t tile_capacity, uint32_t* tile_ranges, void* ws,
                         size_t ws_bytes, void* stream) {
    ws_status s;
    if (n < 0 || n > kMaxGaussians) return fail(WS_ERR_INVALID_ARGUMENT, "n out of range");
    if ((s = check_cameras(cams, d_cams, n_views)) != WS_OK) return s;
    if ((s = check_options(opt)) != WS_OK) return s;
    if (!binned(opt)) return fail(WS_ERR_INVALID_ARGUMENT, "ws_expand_bins needs bins larger than one tile");
    if (int64_t(n) * n_views > kMaxGaussians) return fail(WS_ERR_INVALID_ARGUMENT, "n * n_views must be < 2^31");
    const int64_t per_bin = int64_t(opt->bin_x) * opt->bin_y;
    if (capacity < 0 || capacity > kMaxSortN) return fail(WS_ERR_INVALID_ARGUMENT, "capacity out of range");
    if (tile_capacity < per_bin * capacity || tile_capacity > (int64_t(1) << 32) - 1)
        return fail(WS_ERR_INVALID_ARGUMENT,
                    "tile_capacity must hold bin_x * bin_y * capacity = %lld entries and be below 2^32",
                    (long long)(per_bin * capacity));
    if (capacity > 0 && (!keys || !values || !tile_values))
        return fail(WS_ERR_INVALID_ARGUMENT, "keys / values / tile_values is NULL");
    if (n > 0 && !splats) return fail(WS_ERR_INVALID_ARGUMENT, "splats is NULL");
    if (!d_num_pairs || !d_status || !tile_ranges)
        return fail(WS_ERR_INVALID_ARGUMENT, "d_num_pairs / d_status / tile_ranges is NULL");
    const int64_t bins = total_bins_of(cams, n_views, opt);
    if (bins * per_bin > (int64_t(1) << 31) - 8) return fail(WS_ERR_UNSUPPORTED, "too many tiles");
    if ((s = check_ws(ws, ws_bytes, ws::expand_workspace(bins))) != WS_OK) return s;
    const hipError_t e = ws::launch_expand(splats, n, d_cams, n_views, bins, kopts_for(opt, cams, n_views), keys, values,
                                           capacity, d_num_pairs, d_status, tile_values, tile_ranges, ws,
                                           static_cast<hipStream_t>(stream));
    return hip_status(e, "ws_expand_bins launch");
}

extern "C++" {
namespace {

// The checks and the launch shared by ws_render_backward and ws_render_backward_l1.
ws_status render_backward_checked(const char* name, const ws_gaussians* g, const ws_camera* cams,
                                  const ws_camera* d_cams, int32_t n_views, const ws_options* opt,
                                  const ws_splat* splats, const uint32_t* tiles_touched, const uint32_t* values,
                                  const uint32_t* tile_ranges, const float* images, const float* dL_dimages,
                                  const ws::L1Loss* l1,
                                  const int32_t* d_status,
                                  ws_gaussian_grads* grads, void* ws, size_t ws_bytes, void* stream) {
    ws_status s;
    if ((s = check_gaussians(g)) != WS_OK) return s;
    if ((s = check_cameras(cams, d_cams, n_views)) != WS_OK) return s;
    if ((s = check_options(opt)) != WS_OK) return s;
    if (!grads || (g->n > 0 && (!grads->means || !grads->log_scales || !grads->quats || !grads->opacity_logits ||
                                !grads->sh)))
        return fail(WS_ERR_INVALID_ARGUMENT, "%s: a gradient array is NULL", name);
    if (opt->flags & WS_FLAG_PACKED)
        return fail(WS_ERR_UNSUPPORTED, "%s needs full-precision ws_splat records (no WS_FLAG_PACKED)", name);
    if (!tile_ranges || !images || !d_status)
        return fail(WS_ERR_INVALID_ARGUMENT, "%s: tile_ranges / images / d_status is NULL", name);
    if (!l1 && !dL_dimages) return fail(WS_ERR_INVALID_ARGUMENT, "%s: dL_dimages is NULL", name);
    if (g->n > 0 && (!splats || !values)) return fail(WS_ERR_INVALID_ARGUMENT, "%s: splats / values is NULL", name);
    if (g->n * int64_t(n_views) > kMaxGaussians)
        return fail(WS_ERR_INVALID_ARGUMENT, "%s: n * n_views must be < 2^31", name);
    const int64_t tiles = total_tiles_of(cams, n_views, opt->tile_w, opt->tile_h);
    const size_t need =
        l1 ? ws::render_backward_l1_workspace(g->n, n_views, tiles) : ws::render_backward_workspace(g->n, n_views);
    if ((s = check_ws(ws, ws_bytes, need)) != WS_OK) return s;
    ws::GradPtrs gp;
    gp.means = grads->means;
    gp.log_scales = grads->log_scales;
    gp.quats = grads->quats;
    gp.logits = grads->opacity_logits;
    gp.sh = grads->sh;
    const hipError_t e = ws::launch_render_backward(gauss_ptrs(g), d_cams, n_views, tiles, ws::to_kopts(*opt), splats,
                                                    tiles_touched, values, tile_ranges, images, dL_dimages, d_status, gp, ws,
                                                    static_cast<hipStream_t>(stream), l1);
    return hip_status(e, name);
}

}  // namespace
}  // extern "C++"

ws_status ws_render_backward(const ws_gaussians* g, const ws_camera* cams, const ws_camera* d_cams,
                             int32_t n_views, const ws_options* opt, const ws_splat* splats,
                             const uint32_t* tiles_touched, const uint32_t* values, const uint32_t* tile_ranges,
                             const float* images, const float* dL_dimages, const int32_t* d_status,
                             ws_gaussian_grads* grads, void* ws, size_t ws_bytes, void* stream) {
    return render_backward_checked("ws_render_backward", g, cams, d_cams, n_views, opt, splats, tiles_touched, values,
                                   tile_ranges, images, dL_dimages, nullptr, d_status, grads, ws, ws_bytes, stream);
}

ws_status ws_render_backward_l1(const ws_gaussians* g, const ws_camera* cams, const ws_camera* d_cams,
                                int32_t n_views, const ws_options* opt, const ws_splat* splats,
                                const uint32_t* tiles_touched, const uint32_t* values, const uint32_t* tile_ranges, const float* images,
                                const float* targets, int64_t total, float* d_loss, const int32_t* d_status,
                                ws_gaussian_grads* grads, void* ws, size_t ws_bytes, void* stream) {
    if (!cams || n_views < 1) return fail(WS_ERR_INVALID_ARGUMENT, "ws_render_backward_l1: no cameras");
    int64_t elems = 0;
    for (int32_t v = 0; v < n_views; ++v) elems += 3 * int64_t(cams[v].width) * cams[v].height;
    if (total == 0) total = elems;
    if (total < elems)
        return fail(WS_ERR_INVALID_ARGUMENT, "ws_render_backward_l1: total (%lld) must be 0 or >= the views' %lld "
                    "elements", (long long)total, (long long)elems);
    if (!images || !targets || !d_loss)
        return fail(WS_ERR_INVALID_ARGUMENT, "ws_render_backward_l1: images / targets / d_loss is NULL");
    const ws::L1Loss l1{targets, total, d_loss};
    return render_backward_checked("ws_render_backward_l1", g, cams, d_cams, n_views, opt, splats, tiles_touched,
                                   values, tile_ranges, images, nullptr, &l1, d_status, grads, ws, ws_bytes, stream);
}

ws_status ws_l1_loss(const float* images, const float* targets, int64_t n, int64_t total, float* dL_dimages,
                     float* d_loss, void* ws, size_t ws_bytes, void* stream) {
    if (n < 1) return fail(WS_ERR_INVALID_ARGUMENT, "n must be >= 1");
    if (total == 0) total = n;
    if (total < n)
        return fail(WS_ERR_INVALID_ARGUMENT, "total (%lld) must be 0 or >= n (%lld)", (long long)total, (long long)n);
    if (!images || !targets || !dL_dimages || !d_loss) return fail(WS_ERR_INVALID_ARGUMENT, "a pointer is NULL");
    ws_status s;
    if ((s = check_ws(ws, ws_bytes, ws::l1_loss_workspace(n))) != WS_OK) return s;
    const hipError_t e = ws::launch_l1_loss(images, targets, n, total, dL_dimages, d_loss, ws,
                                          static_cast<hipStream_t>(stream));
    return hip_status(e, "ws_l1_loss launch");
}

struct ws_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

ws_status ws_graph_begin(void* stream) {
    if (!stream) return fail(WS_ERR_INVALID_ARGUMENT, "graph capture needs a non-null stream");
    return hip_status(hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal),
                      "hipStreamBeginCapture");
}

ws_status ws_graph_end(void* stream, ws_graph* out) {
    if (!stream || !out) return fail(WS_ERR_INVALID_ARGUMENT, "stream / out is NULL");
    hipGraph_t g = nullptr;
    ws_status s = hip_status(hipStreamEndCapture(static_cast<hipStream_t>(stream), &g), "hipStreamEndCapture");
    if (s != WS_OK) return s;
    hipGraphExec_t ex = nullptr;
    s = hip_status(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (s != WS_OK) {
        (void)hipGraphDestroy(g);
        return s;
    }
    *out = new ws_graph_s{g, ex};
    return WS_OK;
}

ws_status ws_graph_launch(ws_graph graph, void* stream) {
    if (!graph) return fail(WS_ERR_INVALID_ARGUMENT, "graph is NULL");
    return hip_status(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)), "hipGraphLaunch");
}

ws_status ws_graph_destroy(ws_graph graph) {
    if (!graph) return WS_OK;
    (void)hipGraphExecDestroy(graph->exec);
    (void)hipGraphDestroy(graph->graph);
    delete graph;
    return WS_OK;
}

}  // extern "C"
