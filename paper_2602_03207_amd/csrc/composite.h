// Per-(pixel, splat) compositing arithmetic shared by the forward render and
// its adjoint (Eq. 2 and Eq. 4 with the library's readings):
//   alpha = min(alpha_max, sigma * exp(power)),
//   power = -1/2 (A dx^2 + C dy^2) - B dx dy,  (dx, dy) = mean2d - pixel centre;
//   a splat is skipped where the pixel is outside its rectangle or
//   alpha < alpha_min; the pixel stops before a splat whose compositing would
//   bring the transmittance below t_min; otherwise C += c alpha T, T *= 1 - alpha.
// Evaluation: sigma * exp(power) = 2^(power log2(e) + log2(sigma)), with the
// conic pre-scaled by log2(e) and log2(sigma) computed once when the splat is
// staged, so a (pixel, splat) pair costs one quadratic form and one exp2.
// The transmittance step is T' = fma(-T, alpha, T) and the colour weight is
// T - T' (= alpha T), so the weights of a pixel sum exactly to 1 - T_final.
#pragma once

#include "ws_internal.h"

namespace ws {

constexpr float kLog2e = 1.4426950408889634f;

// A splat staged in LDS for compositing: 48 bytes.
struct StagedSplat {
    float u, v, qa, qb;    // qa = -log2(e)/2 * A, qb = -log2(e) * B
    float qc, ls, r, g;    // qc = -log2(e)/2 * C, ls = log2(sigma)
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
    s.ls = __log2f(r1.y);
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

// sigma * exp(power) for the staged splat (alpha before the clamp):
// 2^(qa dx^2 + dy (qb dx + qc dy) + log2 sigma).
__device__ __forceinline__ float raw_alpha(const StagedSplat& s, float dx, float dy) {
    const float cross = fmaf(s.qb, dx, s.qc * dy);
    const float p2 = fmaf(dy, cross, fmaf(s.qa * dx, dx, s.ls));
    return __builtin_amdgcn_exp2f(p2);
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

// A packed coordinate that lies in no rectangle (real coordinates stay below
// 32768), for lanes without a pixel.
constexpr uint32_t kNoPixel = 0xffffffffu;

struct PixelState {
    uint32_t pxy;  // x | y << 16
    float pcx, pcy;
    float T;
    float c[3];
    int32_t last;  // index (in the tile's list) of the last splat composited, -1 if none

    __device__ __forceinline__ void init(int x, int y) {
        pxy = pack_xy(x, y);
        pcx = float(x) + 0.5f;
        pcy = float(y) + 0.5f;
        T = 1.f;
        c[0] = c[1] = c[2] = 0.f;
        last = -1;
    }
};

// Thresholds of the compositing rule, canonicalised once so that the clamp in
// the inner loop needs no per-iteration canonicalisation.
struct BlendConsts {
    float alpha_min, alpha_max, t_min;
    float log2_amin;  // for the quadrant culling bound only
    __device__ __forceinline__ explicit BlendConsts(const KOpts& o)
        : alpha_min(__builtin_canonicalizef(o.alpha_min)),
          alpha_max(__builtin_canonicalizef(o.alpha_max)),
          t_min(__builtin_canonicalizef(o.t_min)),
          log2_amin(__log2f(o.alpha_min)) {}
};

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ bool lane_in(uint64_t mask) { return __builtin_amdgcn_inverse_ballot_w64(mask); }

// One splat of the list into the pixels of a wave, with the decisions of the
// rule above.  `active` is the wave's set of lanes whose pixel has not stopped
// (a lane mask in scalar registers); the per-lane decisions are formed as lane
// masks too (ballots of the comparisons) and applied with lane_in().  A splat
// that no active lane's rectangle holds changes nothing (all its masks are
// empty), so it needs no separate test.
__device__ __forceinline__ void blend_one(PixelState& ps, uint64_t& active, const StagedSplat& s, int32_t idx,
                                          const BlendConsts& k) {
    const uint64_t inr = active & wave_ballot(in_rect(s, ps.pxy));
    const float dx = s.u - ps.pcx, dy = s.v - ps.pcy;
    // min(alpha_max, sigma e^power) as one clamp: the raw value is never negative
    const float alpha = __builtin_amdgcn_fmed3f(raw_alpha(s, dx, dy), 0.f, k.alpha_max);
    const float Tn = fmaf(-ps.T, alpha, ps.T);
    const uint64_t hit = inr & wave_ballot(!(alpha < k.alpha_min));
    const uint64_t stop = hit & wave_ballot(Tn < k.t_min);
    const bool take = lane_in(hit & ~stop);
    // weight T - T': alpha T where the splat is taken, exactly +0 elsewhere
    // (colours are finite and >= 0, so adding r * 0 leaves the sums unchanged)
    const float T1 = take ? Tn : ps.T;
    const float w = ps.T - T1;
    ps.c[0] = fmaf(s.r, w, ps.c[0]);
    ps.c[1] = fmaf(s.g, w, ps.c[1]);
    ps.c[2] = fmaf(s.b, w, ps.c[2]);
    ps.T = T1;
    ps.last = take ? idx : ps.last;
    active &= ~stop;
}

// ---- pixel layout and per-wave splat lists
//
// A TW x TH tile (both multiples of 8) is split into 8x8 quadrants, one per
// wave: wave w owns quadrant (w % (TW/8), w / (TW/8)) and its lane l the
// pixel (l % 8, l / 8) inside it.  When a batch is staged, every staged splat
// is tested against each quadrant's pixel block; the wave-wide ballots of
// those tests (one 64-bit mask per staging wave and quadrant) let each wave
// walk only the splats whose rectangle meets its quadrant, in list order.

template <int TW>
__device__ __forceinline__ void quadrant_pixel(int x0, int y0, int* px, int* py) {
    const int w = threadIdx.x / kWave, l = int(lane_id());
    *px = x0 + (w % (TW / 8)) * 8 + (l & 7);
    *py = y0 + (w / (TW / 8)) * 8 + (l >> 3);
}

// Can the splat reach alpha >= alpha_min at any pixel centre of the block
// [bx0, bx1] x [by0, by1] (inclusive pixel indices)?  With Q(d) = -(qa dx^2 +
// qb dx dy + qc dy^2) >= 0 the pixel test passes only where Q <= ls -
// log2(alpha_min) =: R.  Q is convex, so its minimum over the box of offsets
// d = mean - pixel centre is 0 when the mean lies in the box and otherwise lies
// on one of the four edges, where it is a one-dimensional quadratic minimised
// in closed form (clamped to the edge).  The answer is "no" only when that
// minimum exceeds R by a margin far above the fp32 rounding of this bound and
// of the per-pixel evaluation (relative to the sizes of the terms involved),
// so a block it rules out holds no pixel whose fp32 alpha reaches alpha_min:
// dropping the splat there changes no pixel and no skip decision.  Non-finite
// values answer "yes".
struct EllipseCull {
    float a, b, c, kx, ky, R, scale;  // Q = a dx^2 + b dx dy + c dy^2
    __device__ __forceinline__ EllipseCull(const StagedSplat& s, float log2_amin) {
        a = -s.qa;
        b = -s.qb;
        c = -s.qc;
        kx = b / (2.f * c);  // edge dx = const: dy* = -kx dx
        ky = b / (2.f * a);  // edge dy = const: dx* = -ky dy
        R = s.ls - log2_amin;
        scale = fabsf(s.ls) + fabsf(log2_amin);
    }
    __device__ __forceinline__ float q(float dx, float dy) const { return fmaf(a * dx, dx, dy * fmaf(b, dx, c * dy)); }
    __device__ __forceinline__ bool meets(const StagedSplat& s, int bx0, int bx1, int by0, int by1) const {
        const float lx0 = s.u - (float(bx1) + 0.5f), lx1 = s.u - (float(bx0) + 0.5f);
        const float ly0 = s.v - (float(by1) + 0.5f), ly1 = s.v - (float(by0) + 0.5f);
        if (lx0 <= 0.f && lx1 >= 0.f && ly0 <= 0.f && ly1 >= 0.f) return true;
        const float q0 = q(lx0, __builtin_amdgcn_fmed3f(-kx * lx0, ly0, ly1));
        const float q1 = q(lx1, __builtin_amdgcn_fmed3f(-kx * lx1, ly0, ly1));
        const float q2 = q(__builtin_amdgcn_fmed3f(-ky * ly0, lx0, lx1), ly0);
        const float q3 = q(__builtin_amdgcn_fmed3f(-ky * ly1, lx0, lx1), ly1);
        const float qmin = fminf(fminf(q0, q1), fminf(q2, q3));
        const float mx = fmaxf(fabsf(lx0), fabsf(lx1)), my = fmaxf(fabsf(ly0), fabsf(ly1));
        const float size = fmaf(a * mx, mx, my * fmaf(fabsf(b), mx, c * my)) + scale;
        const bool finite = __builtin_isfinite(qmin) && __builtin_isfinite(size) && a > 0.f && c > 0.f;
        return !(finite && qmin > R + 1e-4f * size + 1e-4f);
    }
};

// Ballots of "this staged splat meets quadrant q" into masks[q * NW + staging
// wave]: its rectangle meets the quadrant's pixel block and, on the part they
// share, the splat can reach alpha_min (EllipseCull).
template <int TW, int TH>
__device__ __forceinline__ void stage_quadrant_masks(const StagedSplat& s, bool valid, int x0, int y0,
                                                     float log2_amin, uint64_t* masks) {
    constexpr int QX = TW / 8, NQ = (TW / 8) * (TH / 8), NW = TW * TH / kWave;
    const int rx0 = int(s.rxy & 0xffffu), ry0 = int(s.rxy >> 16);
    const int rx1 = rx0 + int(s.rwh & 0xffffu), ry1 = ry0 + int(s.rwh >> 16);
    const int w = threadIdx.x / kWave;
    const EllipseCull ec(s, log2_amin);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int qx0 = x0 + (q % QX) * 8, qy0 = y0 + (q / QX) * 8;
        bool meets = valid && rx0 <= qx0 + 7 && rx1 >= qx0 && ry0 <= qy0 + 7 && ry1 >= qy0;
        if (meets) meets = ec.meets(s, max(rx0, qx0), min(rx1, qx0 + 7), max(ry0, qy0), min(ry1, qy0 + 7));
        const uint64_t b = wave_ballot(meets);
        if (lane_id() == 0) masks[q * NW + w] = b;
    }
}

// The value of lane 0, as a wave-uniform (scalar) value.  readfirstlane
// returns a signed int: each half goes through uint32_t so that the low word
// is not sign-extended into the high one.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v))));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v >> 32))));
    return uint64_t(lo) | (uint64_t(hi) << 32);
}

// The set bits of a wave's NW quadrant masks (held in scalar registers), in
// increasing order (Forward) or decreasing order; next() returns -1 at the end.
template <int NW, bool Forward>
struct MaskWalk {
    uint64_t mk[NW];
    uint64_t m;
    int sw;

    __device__ __forceinline__ void init(const uint64_t* quadrant_masks) {
#pragma unroll
        for (int w = 0; w < NW; ++w) mk[w] = uniform_u64(quadrant_masks[w]);
        sw = Forward ? 0 : NW - 1;
        m = mk[sw];
    }
    __device__ __forceinline__ uint64_t pick(int w) const {
        uint64_t r = mk[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) r = (w == i) ? mk[i] : r;
        return r;
    }
    __device__ __forceinline__ int next() {
        while (m == 0) {
            sw += Forward ? 1 : -1;
            if (sw < 0 || sw >= NW) return -1;
            m = pick(sw);
        }
        const int j = Forward ? __builtin_ctzll(m) : 63 - __builtin_clzll(m);
        m &= ~(uint64_t(1) << j);
        return sw * kWave + j;
    }
};

// Composites, front to back, the staged splats of the batch that meet this
// wave's quadrant (entry j of the batch has index idx0 + j in the tile's
// list): the set bits of the wave's masks, in order, up to four per step with
// all records read from LDS before the first is blended.  The wave leaves once all
// its lanes have stopped (`active` empty); a splat blended after that changes
// nothing.
template <int NW>
__device__ __forceinline__ void composite_batch(PixelState& ps, uint64_t& active, const StagedSplat* batch,
                                                const uint64_t* quadrant_masks, int32_t idx0, const BlendConsts& k) {
    if (active == 0) return;
    uint64_t mk[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) mk[w] = uniform_u64(quadrant_masks[w]);
#pragma unroll
    for (int sw = 0; sw < NW; ++sw) {
        uint64_t m = mk[sw];
        const StagedSplat* wb = batch + sw * kWave;
        const int32_t wi = idx0 + sw * kWave;
        while (m != 0) {
            const int left = __builtin_popcountll(m);
            const int j0 = __builtin_ctzll(m);
            m &= m - 1;
            const StagedSplat s0 = wb[j0];
            if (left >= 4) {
                const int j1 = __builtin_ctzll(m);
                m &= m - 1;
                const int j2 = __builtin_ctzll(m);
                m &= m - 1;
                const int j3 = __builtin_ctzll(m);
                m &= m - 1;
                const StagedSplat s1 = wb[j1], s2 = wb[j2], s3 = wb[j3];
                blend_one(ps, active, s0, wi + j0, k);
                blend_one(ps, active, s1, wi + j1, k);
                blend_one(ps, active, s2, wi + j2, k);
                blend_one(ps, active, s3, wi + j3, k);
            } else if (left >= 2) {
                const int j1 = __builtin_ctzll(m);
                m &= m - 1;
                const StagedSplat s1 = wb[j1];
                blend_one(ps, active, s0, wi + j0, k);
                blend_one(ps, active, s1, wi + j1, k);
            } else {
                blend_one(ps, active, s0, wi + j0, k);
            }
            if (active == 0) return;
        }
    }
}

}  // namespace ws
