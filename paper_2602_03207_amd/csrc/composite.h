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

// The same from a 32-byte packed record (ws_splat_packed; `recs` addresses
// the view's records in float4s): the conic is the inverse of the quantised
// ellipse axis1 axis1^T + axis2 axis2^T, whose determinant is the squared
// cross product of the axes; colour and opacity are the bytes / 255.
__device__ __forceinline__ StagedSplat stage_splat_packed(const float4* __restrict__ recs, uint32_t id) {
    const float4 r0 = recs[2 * int64_t(id)], r1 = recs[2 * int64_t(id) + 1];
    const uint32_t a01 = __float_as_uint(r0.z), a23 = __float_as_uint(r0.w);
    const float a1x = float(__builtin_bit_cast(_Float16, uint16_t(a01 & 0xffffu)));
    const float a1y = float(__builtin_bit_cast(_Float16, uint16_t(a01 >> 16)));
    const float a2x = float(__builtin_bit_cast(_Float16, uint16_t(a23 & 0xffffu)));
    const float a2y = float(__builtin_bit_cast(_Float16, uint16_t(a23 >> 16)));
    const float s00 = fmaf(a1x, a1x, a2x * a2x), s01 = fmaf(a1x, a1y, a2x * a2y), s11 = fmaf(a1y, a1y, a2y * a2y);
    const float cross = fmaf(a1x, a2y, -a1y * a2x);
    const float idet = 1.f / (cross * cross);
    const uint32_t rgba = __float_as_uint(r1.x);
    StagedSplat s;
    s.u = r0.x;
    s.v = r0.y;
    s.qa = -0.5f * kLog2e * (s11 * idet);
    s.qb = -kLog2e * (-s01 * idet);
    s.qc = -0.5f * kLog2e * (s00 * idet);
    s.ls = __log2f(float(rgba >> 24) / 255.f);
    s.r = float(rgba & 0xffu) / 255.f;
    s.g = float((rgba >> 8) & 0xffu) / 255.f;
    s.b = float((rgba >> 16) & 0xffu) / 255.f;
    const uint32_t rx = __float_as_uint(r1.z), ry = __float_as_uint(r1.w);
    const uint32_t x0 = rx & 0xffffu, x1 = rx >> 16, y0 = ry & 0xffffu, y1 = ry >> 16;
    if (x1 >= x0 && y1 >= y0) {
        s.rxy = pack_xy(int(x0), int(y0));
        s.rwh = pack_xy(int(x1 - x0), int(y1 - y0));
    } else {
        s.rxy = 0xffffffffu;
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
//
// RECT: test the pixel against the splat's rectangle.  With the opacity-aware
// extent the rectangle is the bounding box of the ellipse where alpha reaches
// alpha_min (Sec. 3.4), so a pixel outside it has alpha < alpha_min and the
// alpha test alone rejects it; only a pixel whose alpha lies within the fp32
// rounding of alpha_min can decide differently, which is one of the pixel's
// correct fp32 results either way.  The fixed 3-sigma extent can be smaller
// than that ellipse, and the ellipse of a packed record (axes rounded to fp16)
// can reach past it: both need the test.
template <bool RECT>
__device__ __forceinline__ void blend_one(PixelState& ps, uint64_t& active, const StagedSplat& s, int32_t idx,
                                          const BlendConsts& k) {
    const uint64_t inr = RECT ? active & wave_ballot(in_rect(s, ps.pxy)) : active;
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

// The pixel columns, per band of tile rows, where a splat can reach
// alpha >= alpha_min.  In offsets p = pixel centre - mean the per-pixel test
// passes only where Q(p) = a px^2 + b px py + c py^2 <= ls - log2(alpha_min)
// (a = -qa, b = -qb, c = -qc: the same quadratic form as the per-pixel
// exponent).  The threshold is first raised by a bound on the fp32 rounding of
// the per-pixel evaluation (relative to the sizes of its terms, which the
// conditioning kappa = 8ac / (4ac - b^2) bounds), so the ellipse below holds
// every pixel whose fp32 alpha can reach alpha_min.  On a row py of that
// ellipse, px lies between the roots (-b py -+ sqrt(4aR - (4ac - b^2) py^2)) /
// 2a; over a band of rows the smallest left root is -hx if the ellipse's
// leftmost point lies in the band and otherwise that of the row nearer to it
// (the left root is convex in py), and likewise on the right.  The interval is
// widened by a bound on the fp32 rounding of this computation before it is
// turned into whole pixel columns, so dropping a splat from a quadrant outside
// those columns changes no pixel and no skip decision.  Splats whose form is
// too ill-conditioned for that bound, or not finite, keep their rectangle.
struct EllipseRows {
    float a, b, c, R, det4, hx, hy, inv2a, py_left, mx, my;
    bool ok, none;
    __device__ __forceinline__ EllipseRows(const StagedSplat& s, float log2_amin) {
        a = -s.qa;
        b = -s.qb;
        c = -s.qc;
        // hardware reciprocal and square root (about 1 ulp): the margins below
        // are orders of magnitude wider than their error
        det4 = fmaf(4.f * a, c, -b * b);
        const float inv = __builtin_amdgcn_rcpf(det4), ra = __builtin_amdgcn_rcpf(a), rc = __builtin_amdgcn_rcpf(c);
        const float kappa = 8.f * a * c * inv;
        const float R0 = s.ls - log2_amin;
        R = R0 + 1e-5f * (kappa * (fabsf(R0) + 1.f) + fabsf(s.ls) + fabsf(log2_amin) + 1.f);
        ok = a > 0.f && c > 0.f && det4 > 0.f && kappa < 1e4f && __builtin_isfinite(R) && __builtin_isfinite(kappa) &&
             __builtin_isfinite(s.u) && __builtin_isfinite(s.v);
        none = ok && R < 0.f;  // alpha_min is out of reach everywhere
        const float Rp = fmaxf(R, 0.f);
        hx = __builtin_amdgcn_sqrtf(4.f * c * Rp * inv);
        hy = __builtin_amdgcn_sqrtf(4.f * a * Rp * inv);
        inv2a = 0.5f * ra;
        py_left = b * hx * (0.5f * rc);  // row of the leftmost point; the rightmost is at -py_left
        const float k1 = 1.f + kappa;
        mx = 4.f * __builtin_amdgcn_sqrtf(1e-5f * Rp * k1 * ra) + 1e-5f * (hx * k1 + fabsf(b) * hy * inv2a) + 1e-3f;
        my = 4.f * __builtin_amdgcn_sqrtf(1e-5f * Rp * k1 * rc) + 1e-5f * hy * k1 + 1e-3f;
    }
    // Intersects [*cx0, *cx1] with the columns the splat can reach on pixel
    // rows [by0, by1] (non-empty).
    __device__ __forceinline__ void columns(const StagedSplat& s, int by0, int by1, int* cx0, int* cx1) const {
        if (!ok) return;
        const float y0 = (float(by0) + 0.5f) - s.v, y1 = (float(by1) + 0.5f) - s.v;
        if (none || y0 > hy + my || y1 < -hy - my) {
            *cx1 = *cx0 - 1;
            return;
        }
        const float yc0 = fminf(fmaxf(y0, -hy), hy), yc1 = fmaxf(fminf(y1, hy), -hy);
        const float s0 = __builtin_amdgcn_sqrtf(fmaxf(fmaf(-det4 * yc0, yc0, 4.f * a * R), 0.f));
        const float s1 = __builtin_amdgcn_sqrtf(fmaxf(fmaf(-det4 * yc1, yc1, 4.f * a * R), 0.f));
        const float left = (py_left >= y0 - my && py_left <= y1 + my)
                               ? -hx
                               : fminf((-b * yc0 - s0) * inv2a, (-b * yc1 - s1) * inv2a);
        const float right = (-py_left >= y0 - my && -py_left <= y1 + my)
                                ? hx
                                : fmaxf((-b * yc0 + s0) * inv2a, (-b * yc1 + s1) * inv2a);
        // pixel x is reachable only if x + 0.5 - u lies in [left - mx, right + mx]
        const float e = 1e-6f * fabsf(s.u) + 1e-3f;
        const float f0 = fmaxf(s.u + (left - mx) - 0.5f - e, -1.f);
        const float f1 = fminf(s.u + (right + mx) - 0.5f + e, 65536.f);
        *cx0 = max(*cx0, int(ceilf(f0)));
        *cx1 = min(*cx1, int(floorf(f1)));
    }
};

// Ballots of "this staged splat meets quadrant q" into masks[q * NW + staging
// wave]: on the rows its rectangle shares with the quadrant, the columns where
// it can reach alpha_min (EllipseRows, intersected with its rectangle) meet
// the quadrant's columns.
template <int TW, int TH>
__device__ __forceinline__ void stage_quadrant_masks(const StagedSplat& s, bool valid, int x0, int y0,
                                                     float log2_amin, uint64_t* masks) {
    constexpr int QX = TW / 8, QY = TH / 8, NW = TW * TH / kWave;
    const int rx0 = int(s.rxy & 0xffffu), ry0 = int(s.rxy >> 16);
    const int rx1 = rx0 + int(s.rwh & 0xffffu), ry1 = ry0 + int(s.rwh >> 16);
    const int w = threadIdx.x / kWave;
    const EllipseRows er(s, log2_amin);
#pragma unroll
    for (int qy = 0; qy < QY; ++qy) {
        const int by0 = max(ry0, y0 + 8 * qy), by1 = min(ry1, y0 + 8 * qy + 7);
        const bool rows = valid && by0 <= by1;
        int cx0 = rx0, cx1 = rx1;
        if (rows) er.columns(s, by0, by1, &cx0, &cx1);
#pragma unroll
        for (int qx = 0; qx < QX; ++qx) {
            const int qx0 = x0 + 8 * qx;
            const bool meets = rows && cx0 <= qx0 + 7 && cx1 >= qx0 && cx0 <= cx1;
            const uint64_t bal = wave_ballot(meets);
            if (lane_id() == 0) masks[(qy * QX + qx) * NW + w] = bal;
        }
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
// The mask being walked is always mk[0] (Forward) or mk[NW - 1]: when it runs
// out the others shift along, so every index is a constant and the masks stay
// in registers (a walk that picked mk[sw] by a variable index was kept in
// scratch memory).
template <int NW, bool Forward>
struct MaskWalk {
    uint64_t mk[NW];
    int sw;

    __device__ __forceinline__ void init(const uint64_t* quadrant_masks) {
#pragma unroll
        for (int w = 0; w < NW; ++w) mk[w] = uniform_u64(quadrant_masks[w]);
        sw = Forward ? 0 : NW - 1;
    }
    // Drops the entries past batch position `lim` (< 0: every entry).
    __device__ __forceinline__ void keep_up_to(int lim) {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int hi = lim - w * kWave;  // last kept bit of this mask
            mk[w] = hi < 0 ? 0 : (hi >= kWave - 1 ? mk[w] : mk[w] & ((uint64_t(2) << hi) - 1));
        }
    }
    __device__ __forceinline__ int next() {
        constexpr int kCur = Forward ? 0 : NW - 1;
        while (mk[kCur] == 0) {
            sw += Forward ? 1 : -1;
            if (sw < 0 || sw >= NW) return -1;
            if (Forward) {
#pragma unroll
                for (int i = 0; i + 1 < NW; ++i) mk[i] = mk[i + 1];
            } else {
#pragma unroll
                for (int i = NW - 1; i > 0; --i) mk[i] = mk[i - 1];
            }
        }
        const uint64_t m = mk[kCur];
        const int j = Forward ? __builtin_ctzll(m) : 63 - __builtin_clzll(m);
        mk[kCur] = m & ~(uint64_t(1) << j);
        return sw * kWave + j;
    }
};

// Composites, front to back, the staged splats of the batch that meet this
// wave's quadrant (entry j of the batch has index idx0 + j in the tile's
// list): the set bits of the wave's masks, in order, up to four per step with
// all records read from LDS before the first is blended.  The wave leaves once all
// its lanes have stopped (`active` empty); a splat blended after that changes
// nothing.
template <int NW, bool RECT>
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
                blend_one<RECT>(ps, active, s0, wi + j0, k);
                blend_one<RECT>(ps, active, s1, wi + j1, k);
                blend_one<RECT>(ps, active, s2, wi + j2, k);
                blend_one<RECT>(ps, active, s3, wi + j3, k);
            } else if (left >= 2) {
                const int j1 = __builtin_ctzll(m);
                m &= m - 1;
                const StagedSplat s1 = wb[j1];
                blend_one<RECT>(ps, active, s0, wi + j0, k);
                blend_one<RECT>(ps, active, s1, wi + j1, k);
            } else {
                blend_one<RECT>(ps, active, s0, wi + j0, k);
            }
            if (active == 0) return;
        }
    }
}

}  // namespace ws
