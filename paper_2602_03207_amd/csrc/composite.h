// Per-(pixel, splat) compositing arithmetic shared by the forward render and
// its adjoint (Eq. 2 and Eq. 4 with the library's readings):
//   alpha = min(alpha_max, sigma * exp(power)),
//   power = -1/2 (A dx^2 + C dy^2) - B dx dy,  (dx, dy) = mean2d - pixel centre;
//   a splat is skipped where the pixel is outside its rectangle or
//   alpha < alpha_min; the pixel stops before a splat whose compositing would
//   bring the transmittance below t_min; otherwise C += c alpha T, T *= 1 - alpha.
// The exponential is evaluated as exp2 with the conic pre-scaled by log2(e)
// when the splat is staged, which folds one multiply out of the inner loop.
#pragma once

#include "ws_internal.h"

namespace ws {

constexpr float kLog2e = 1.4426950408889634f;

// A splat staged in LDS for compositing: 48 bytes.
struct StagedSplat {
    float u, v, qa, qb;    // qa = -log2(e)/2 * A, qb = -log2(e) * B
    float qc, sigma, r, g; // qc = -log2(e)/2 * C
    float b;
    uint32_t rxy;          // x0 | y0 << 16: first pixel of the inclusive rectangle
    uint32_t rwh;          // (x1 - x0) | (y1 - y0) << 16
    uint32_t id;           // Gaussian id
};

// Two 16-bit lanes packed in one register (pixel or rectangle coordinates).
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_xy(int x, int y) { return uint32_t(x) | (uint32_t(y) << 16); }

__device__ __forceinline__ StagedSplat stage_splat(const ws_splat* __restrict__ vsplats, uint32_t id) {
    const float4* rec = reinterpret_cast<const float4*>(vsplats + id);
    const float4 r0 = rec[0], r1 = rec[1], r2 = rec[2];
    StagedSplat s;
    s.u = r0.x;
    s.v = r0.y;
    s.qa = -0.5f * kLog2e * r0.z;
    s.qb = -kLog2e * r0.w;
    s.qc = -0.5f * kLog2e * r1.x;
    s.sigma = r1.y;
    s.r = r1.z;
    s.g = r1.w;
    s.b = r2.x;
    const uint32_t rx = __float_as_uint(r2.z), ry = __float_as_uint(r2.w);  // x0 | x1 << 16, y0 | y1 << 16
    const uint32_t x0 = rx & 0xffffu, x1 = rx >> 16, y0 = ry & 0xffffu, y1 = ry >> 16;
    if (x1 >= x0 && y1 >= y0) {
        s.rxy = pack_xy(int(x0), int(y0));
        s.rwh = pack_xy(int(x1 - x0), int(y1 - y0));
    } else {
        s.rxy = 0xffffffffu;  // holds no pixel (coordinates stay below 32768)
        s.rwh = 0u;
    }
    s.id = id;
    return s;
}

// A splat that covers no pixel: used for out-of-range ids.
__device__ __forceinline__ StagedSplat empty_splat() {
    StagedSplat s{};
    s.rxy = 0xffffffffu;
    s.rwh = 0u;
    return s;
}

// Pixel pxy = x | y << 16 inside the splat's rectangle: per 16-bit lane,
// (p - first) mod 2^16 <= extent; both tests in two packed integer ops.
__device__ __forceinline__ bool in_rect(const StagedSplat& s, uint32_t pxy) {
    const u16x2 d = __builtin_bit_cast(u16x2, pxy) - __builtin_bit_cast(u16x2, s.rxy);
    const u16x2 m = __builtin_elementwise_min(d, __builtin_bit_cast(u16x2, s.rwh));
    return __builtin_bit_cast(uint32_t, m) == __builtin_bit_cast(uint32_t, d);
}

// exp(power) for the staged conic; returns sigma * exp(power) (before the clamp).
__device__ __forceinline__ float raw_alpha(const StagedSplat& s, float dx, float dy, float* G) {
    const float p2 = fmaf(s.qa * dx, dx, fmaf(s.qc * dy, dy, s.qb * dx * dy));
    const float e = __builtin_amdgcn_exp2f(p2);
    *G = e;
    return s.sigma * e;
}

struct TileInfo {
    int32_t view, W, H, x0, y0;
    int64_t img_off;
};

// Which view and which pixel block a global tile id names.
__device__ __forceinline__ TileInfo locate_tile(const ws_camera* cams, int32_t n_views, int64_t g, int TW, int TH) {
    int64_t toff = 0, ioff = 0;
    int32_t v = 0;
    int32_t W = cams[0].width, H = cams[0].height;
    for (; v < n_views; ++v) {
        W = cams[v].width;
        H = cams[v].height;
        const int64_t nt = int64_t(ceil_div(W, TW)) * ceil_div(H, TH);
        if (g < toff + nt) break;
        toff += nt;
        ioff += 3ll * W * H;
    }
    const int32_t tiles_x = ceil_div(W, TW);
    const int32_t local = int32_t(g - toff);
    const int32_t ty = local / tiles_x, tx = local - ty * tiles_x;
    TileInfo t;
    t.view = v;
    t.W = W;
    t.H = H;
    t.x0 = tx * TW;
    t.y0 = ty * TH;
    t.img_off = ioff;
    return t;
}

struct PixelState {
    uint32_t pxy;  // x | y << 16
    float pcx, pcy;
    float T;
    float c[3];
    bool done;
    int32_t last;  // index (in the tile's list) of the last splat composited, -1 if none

    __device__ __forceinline__ void init(int x, int y, bool finished) {
        pxy = pack_xy(x, y);
        pcx = float(x) + 0.5f;
        pcy = float(y) + 0.5f;
        T = 1.f;
        c[0] = c[1] = c[2] = 0.f;
        done = finished;
        last = -1;
    }
};

// One splat of the list into one pixel, with the decisions of the rule above.
// Returns true once no lane of the wave is left active.
__device__ __forceinline__ bool blend_one(PixelState& ps, const StagedSplat& s, int32_t idx, const KOpts& o) {
    const bool inr = in_rect(s, ps.pxy) & !ps.done;
    if (__ballot(inr) == 0) return false;  // the whole wave skips this splat
    const float dx = s.u - ps.pcx, dy = s.v - ps.pcy;
    float G;
    const float alpha = fminf(o.alpha_max, raw_alpha(s, dx, dy, &G));
    const float Tn = ps.T * (1.f - alpha);
    const bool hit = inr & !(alpha < o.alpha_min);
    const bool stop = hit & (Tn < o.t_min);
    const bool take = hit & !stop;
    const float w = alpha * ps.T;
    ps.c[0] = take ? fmaf(s.r, w, ps.c[0]) : ps.c[0];
    ps.c[1] = take ? fmaf(s.g, w, ps.c[1]) : ps.c[1];
    ps.c[2] = take ? fmaf(s.b, w, ps.c[2]) : ps.c[2];
    ps.T = take ? Tn : ps.T;
    ps.last = take ? idx : ps.last;
    if (__ballot(stop) == 0) return false;
    ps.done = ps.done | stop;
    return __ballot(!ps.done) == 0;
}

// Composites the staged splats batch[0, cnt) (cnt >= 1), whose first entry has
// index idx0 in the tile's list, front to back.  Two records alternate in
// registers so that the next one is read from LDS while the current one is
// blended; the wave leaves once all its lanes have stopped.
__device__ __forceinline__ void composite_batch(PixelState& ps, const StagedSplat* batch, int cnt, int32_t idx0,
                                                const KOpts& o) {
    if (__ballot(!ps.done) == 0) return;
    StagedSplat s0 = batch[0], s1;
    int j = 0;
    while (true) {
        s1 = batch[j + 1 < cnt ? j + 1 : j];
        if (blend_one(ps, s0, idx0 + j, o) || ++j >= cnt) return;
        s0 = batch[j + 1 < cnt ? j + 1 : j];
        if (blend_one(ps, s1, idx0 + j, o) || ++j >= cnt) return;
    }
}

}  // namespace ws
