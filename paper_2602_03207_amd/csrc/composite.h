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
    uint32_t rx, ry;       // x0 | x1 << 16, y0 | y1 << 16 (inclusive pixel rectangle)
    uint32_t id;           // Gaussian id
};

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
    s.rx = __float_as_uint(r2.z);
    s.ry = __float_as_uint(r2.w);
    s.id = id;
    return s;
}

// A splat that covers no pixel (x0 > x1): used for out-of-range ids.
__device__ __forceinline__ StagedSplat empty_splat() {
    StagedSplat s{};
    s.rx = 1u;  // x0 = 1, x1 = 0
    s.ry = 1u;
    return s;
}

__device__ __forceinline__ bool in_rect(const StagedSplat& s, int px, int py) {
    const uint32_t x0 = s.rx & 0xffffu, x1 = s.rx >> 16, y0 = s.ry & 0xffffu, y1 = s.ry >> 16;
    return uint32_t(px - int(x0)) <= x1 - x0 && uint32_t(py - int(y0)) <= y1 - y0;
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
    int px, py;
    float pcx, pcy;
    float T;
    float c[3];
    bool done;
    int32_t last;   // index (in the tile's list) of the last splat composited, -1 if none
    int32_t count;  // list entries consumed so far

    __device__ __forceinline__ void init(int x, int y, bool finished) {
        px = x;
        py = y;
        pcx = float(x) + 0.5f;
        pcy = float(y) + 0.5f;
        T = 1.f;
        c[0] = c[1] = c[2] = 0.f;
        done = finished;
        last = -1;
        count = 0;
    }

    // Composite one splat; returns true once the pixel has stopped.
    __device__ __forceinline__ bool step(const StagedSplat& s, const KOpts& o) {
        const int32_t idx = count++;
        if (!in_rect(s, px, py)) return false;
        const float dx = s.u - pcx, dy = s.v - pcy;
        float G;
        const float alpha = fminf(o.alpha_max, raw_alpha(s, dx, dy, &G));
        if (alpha < o.alpha_min) return false;
        const float Tn = T * (1.f - alpha);
        if (Tn < o.t_min) {
            done = true;
            return true;
        }
        const float w = alpha * T;
        c[0] = fmaf(s.r, w, c[0]);
        c[1] = fmaf(s.g, w, c[1]);
        c[2] = fmaf(s.b, w, c[2]);
        T = Tn;
        last = idx;
        return false;
    }
};

}  // namespace ws
