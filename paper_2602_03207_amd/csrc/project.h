// Per-(view, Gaussian) projection on the GPU: EWA projection of the 3D
// covariance (Sec. 2.1, Eq. 1-2), view-dependent SH colour (Eq. 3) and the
// opacity-aware bounding box (Sec. 3.4, Eq. 7-8).  The forward preprocess
// and its adjoint both call compute_projection() so that they take the
// same discrete decisions.
//
// Precision: the camera-space centre p = R X + t is formed in fp64 (the
// products of two fp32 values are exact there, so the fp32 depth key is the
// correctly rounded depth); everything else is fp32.
#pragma once

#include "ws_internal.h"

namespace ws {

// Real SH basis constants (orthonormal on the sphere), l <= 3.
constexpr float kSH0 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
constexpr float kSH1 = 0.48860251190291992f;   // sqrt(3 / (4 pi))
constexpr float kSH2a = 1.0925484305920792f;   // sqrt(15 / pi) / 2
constexpr float kSH2b = 0.31539156525252005f;  // sqrt(5 / pi) / 4
constexpr float kSH2c = 0.54627421529603959f;  // sqrt(15 / pi) / 4
constexpr float kSH3a = 0.59004358992664352f;  // sqrt(35 / (2 pi)) / 4
constexpr float kSH3b = 2.8906114426405538f;   // sqrt(105 / pi) / 2
constexpr float kSH3c = 0.45704579946446572f;  // sqrt(21 / (2 pi)) / 4
constexpr float kSH3d = 0.37317633259011546f;  // sqrt(7 / pi) / 4
constexpr float kSH3e = 1.4453057213202769f;   // sqrt(105 / pi) / 4

// SH basis at unit direction (x, y, z) with the Condon-Shortley phase
// (odd-|m| terms negated), index k = l^2 + l + m.
__device__ __forceinline__ void sh_eval_basis(float x, float y, float z, int degree, float* Y) {
    Y[0] = kSH0;
    if (degree < 1) return;
    Y[1] = -kSH1 * y;
    Y[2] = kSH1 * z;
    Y[3] = -kSH1 * x;
    if (degree < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kSH2a * x * y;
    Y[5] = -kSH2a * y * z;
    Y[6] = kSH2b * (2.f * zz - xx - yy);
    Y[7] = -kSH2a * x * z;
    Y[8] = kSH2c * (xx - yy);
    if (degree < 3) return;
    Y[9] = -kSH3a * y * (3.f * xx - yy);
    Y[10] = kSH3b * x * y * z;
    Y[11] = -kSH3c * y * (4.f * zz - xx - yy);
    Y[12] = kSH3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
    Y[13] = -kSH3c * x * (4.f * zz - xx - yy);
    Y[14] = kSH3e * z * (xx - yy);
    Y[15] = -kSH3a * x * (xx - 3.f * yy);
}

// Gradient of sum_k w[k] Y_k(x, y, z) with respect to (x, y, z), treating
// the basis polynomials as functions of three independent variables.
__device__ __forceinline__ void sh_basis_vjp(float x, float y, float z, int degree, const float* w, float* gx,
                                             float* gy, float* gz) {
    float ax = 0.f, ay = 0.f, az = 0.f;
    if (degree >= 1) {
        ay += -kSH1 * w[1];
        az += kSH1 * w[2];
        ax += -kSH1 * w[3];
    }
    if (degree >= 2) {
        ax += kSH2a * y * w[4];
        ay += kSH2a * x * w[4];
        ay += -kSH2a * z * w[5];
        az += -kSH2a * y * w[5];
        ax += -2.f * kSH2b * x * w[6];
        ay += -2.f * kSH2b * y * w[6];
        az += 4.f * kSH2b * z * w[6];
        ax += -kSH2a * z * w[7];
        az += -kSH2a * x * w[7];
        ax += 2.f * kSH2c * x * w[8];
        ay += -2.f * kSH2c * y * w[8];
    }
    if (degree >= 3) {
        const float xx = x * x, yy = y * y, zz = z * z;
        // Y9 = -a y (3xx - yy)
        ax += -kSH3a * 6.f * x * y * w[9];
        ay += -kSH3a * (3.f * xx - 3.f * yy) * w[9];
        // Y10 = b x y z
        ax += kSH3b * y * z * w[10];
        ay += kSH3b * x * z * w[10];
        az += kSH3b * x * y * w[10];
        // Y11 = -c y (4zz - xx - yy)
        ax += -kSH3c * y * (-2.f * x) * w[11];
        ay += -kSH3c * (4.f * zz - xx - 3.f * yy) * w[11];
        az += -kSH3c * y * 8.f * z * w[11];
        // Y12 = d z (2zz - 3xx - 3yy)
        ax += kSH3d * z * (-6.f * x) * w[12];
        ay += kSH3d * z * (-6.f * y) * w[12];
        az += kSH3d * (6.f * zz - 3.f * xx - 3.f * yy) * w[12];
        // Y13 = -c x (4zz - xx - yy)
        ax += -kSH3c * (4.f * zz - 3.f * xx - yy) * w[13];
        ay += -kSH3c * x * (-2.f * y) * w[13];
        az += -kSH3c * x * 8.f * z * w[13];
        // Y14 = e z (xx - yy)
        ax += kSH3e * z * 2.f * x * w[14];
        ay += kSH3e * z * (-2.f * y) * w[14];
        az += kSH3e * (xx - yy) * w[14];
        // Y15 = -a x (xx - 3yy)
        ax += -kSH3a * (3.f * xx - 3.f * yy) * w[15];
        ay += -kSH3a * x * (-6.f * y) * w[15];
    }
    *gx = ax;
    *gy = ay;
    *gz = az;
}

constexpr uint32_t kClampR = 1u, kClampG = 2u, kClampB = 4u, kClampJx = 8u, kClampJy = 16u;

// Everything the forward needs, and the intermediates the adjoint reuses.
struct ProjState {
    bool alive;        // passes the opacity test
    bool visible;      // emits at least one tile
    float sigma;
    double px, py, pz;  // camera-space centre
    float z32, invz;
    float rxc, ryc;     // clamped x/z, y/z used by the Jacobian
    uint32_t clamp;     // kClamp* bits
    float q[4];         // normalised quaternion
    float qnorm;
    float Rq[9];
    float s[3];         // scales
    float T[9];         // W Rq (camera rotation times Gaussian rotation)
    float M[6];         // 2x3 = J W Rq S
    float a, b, c;      // Sigma' entries incl. lowpass
    float det;
    float u, v;
    float A, B, C;      // conic
    float rgb[3];
    float dir[3];       // unit view direction
    float dir_norm;
    uint16_t rect[4];
    uint32_t tiles;
};

__device__ __forceinline__ bool finitef(float x) { return __builtin_isfinite(x); }

// Geometry and colour of Gaussian i for camera `cam`, SH degree DEG (equal to
// o.sh_degree).  Returns st.visible.  With COLOUR false the view-dependent
// colour (and its finiteness test) is skipped: for callers that need the
// geometry of a splat already known to be visible.
template <int DEG, bool COLOUR = true>
__device__ __forceinline__ bool compute_projection(const GaussPtrs& g, int64_t i, const ws_camera& cam,
                                                   const KOpts& o, ProjState& st) {
    const int64_t n = g.n;
    st.alive = false;
    st.visible = false;
    st.tiles = 0;
    st.clamp = 0;
    const float logit = g.logits[i];
    st.sigma = 1.f / (1.f + expf(-logit));
    // opacity cull first: a culled lane issues no further loads
    if (!(st.sigma >= o.alpha_min) || !finitef(logit)) return false;
    const float mx = g.means[i], my = g.means[n + i], mz = g.means[2 * n + i];
    if (!(finitef(mx) && finitef(my) && finitef(mz))) return false;
    // camera-space centre in fp64: products of fp32 values are exact, so the
    // fp32 rounding of z is the correctly rounded depth.
    const double dmx = mx, dmy = my, dmz = mz;
    st.px = ((double(cam.R[0]) * dmx + double(cam.R[1]) * dmy) + double(cam.R[2]) * dmz) + double(cam.t[0]);
    st.py = ((double(cam.R[3]) * dmx + double(cam.R[4]) * dmy) + double(cam.R[5]) * dmz) + double(cam.t[1]);
    st.pz = ((double(cam.R[6]) * dmx + double(cam.R[7]) * dmy) + double(cam.R[8]) * dmz) + double(cam.t[2]);
    if (!(st.pz > double(o.near_z))) return false;
    st.alive = true;
    const float ls0 = g.log_scales[i], ls1 = g.log_scales[n + i], ls2 = g.log_scales[2 * n + i];
    const float q0 = g.quats[i], q1 = g.quats[n + i], q2 = g.quats[2 * n + i], q3 = g.quats[3 * n + i];
    if (!(finitef(ls0) && finitef(ls1) && finitef(ls2) && finitef(q0) && finitef(q1) && finitef(q2) && finitef(q3)))
        return false;
    const float qq = q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
    if (!(qq > 0.f)) return false;
    st.z32 = float(st.pz);
    const double inv_z = 1.0 / st.pz;
    const double rx = st.px * inv_z, ry = st.py * inv_z;
    st.u = float(double(cam.fx) * rx + double(cam.cx));
    st.v = float(double(cam.fy) * ry + double(cam.cy));
    st.invz = float(inv_z);

    // Gaussian rotation and scale
    st.qnorm = sqrtf(qq);
    const float iq = 1.f / st.qnorm;
    const float w = q0 * iq, x = q1 * iq, y = q2 * iq, z = q3 * iq;
    st.q[0] = w; st.q[1] = x; st.q[2] = y; st.q[3] = z;
    float* Rq = st.Rq;
    Rq[0] = 1.f - 2.f * (y * y + z * z); Rq[1] = 2.f * (x * y - w * z);       Rq[2] = 2.f * (x * z + w * y);
    Rq[3] = 2.f * (x * y + w * z);       Rq[4] = 1.f - 2.f * (x * x + z * z); Rq[5] = 2.f * (y * z - w * x);
    Rq[6] = 2.f * (x * z - w * y);       Rq[7] = 2.f * (y * z + w * x);       Rq[8] = 1.f - 2.f * (x * x + y * y);
    st.s[0] = expf(ls0); st.s[1] = expf(ls1); st.s[2] = expf(ls2);
    // T = W Rq
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
            st.T[r * 3 + cc] = cam.R[r * 3 + 0] * Rq[0 * 3 + cc] + cam.R[r * 3 + 1] * Rq[1 * 3 + cc] +
                               cam.R[r * 3 + 2] * Rq[2 * 3 + cc];
    // Jacobian of the projection at the (clamped) centre
    const float limx = o.clamp_fov * (0.5f * float(cam.width) / cam.fx);
    const float limy = o.clamp_fov * (0.5f * float(cam.height) / cam.fy);
    float rxf = float(rx), ryf = float(ry);
    if (rxf > limx) { rxf = limx; st.clamp |= kClampJx; }
    if (rxf < -limx) { rxf = -limx; st.clamp |= kClampJx; }
    if (ryf > limy) { ryf = limy; st.clamp |= kClampJy; }
    if (ryf < -limy) { ryf = -limy; st.clamp |= kClampJy; }
    st.rxc = rxf; st.ryc = ryf;
    const float j00 = cam.fx * st.invz, j02 = -cam.fx * rxf * st.invz;
    const float j11 = cam.fy * st.invz, j12 = -cam.fy * ryf * st.invz;
    // M = J (W Rq S), 2x3
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        st.M[cc] = (j00 * st.T[0 * 3 + cc] + j02 * st.T[2 * 3 + cc]) * st.s[cc];
        st.M[3 + cc] = (j11 * st.T[1 * 3 + cc] + j12 * st.T[2 * 3 + cc]) * st.s[cc];
    }
    const float* M = st.M;
    const float r0 = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    const float r1 = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    const float lp = o.lowpass;
    st.a = r0 + lp;
    st.b = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    st.c = r1 + lp;
    // det(M M^T + lp I) by Cauchy-Binet: sum of squared 2x2 minors of M plus
    // lp * trace + lp^2; no cancellation for needle-shaped splats.
    const float m01 = fmaf(M[0], M[4], -M[1] * M[3]);
    const float m02 = fmaf(M[0], M[5], -M[2] * M[3]);
    const float m12 = fmaf(M[1], M[5], -M[2] * M[4]);
    st.det = (m01 * m01 + m02 * m02 + m12 * m12) + lp * (r0 + r1) + lp * lp;
    if (!(st.det > 0.f) || !finitef(st.det) || !finitef(st.u) || !finitef(st.v)) { st.alive = false; return false; }
    const float idet = 1.f / st.det;
    st.A = st.c * idet;
    st.B = -st.b * idet;
    st.C = st.a * idet;

    // Opacity-aware extent: alpha = sigma e^{-m^2/2} reaches alpha_min at m^2 = 2 ln(sigma / alpha_min).
    const float d2 = (o.flags & WS_FLAG_FIXED_3SIGMA) ? 9.f : 2.f * logf(st.sigma / o.alpha_min);
    const float hx = sqrtf(d2 * st.a), hy = sqrtf(d2 * st.c);
    // pixel i is covered iff u - hx - 0.5 <= i <= u + hx - 0.5
    float x0 = ceilf(st.u - hx - 0.5f), x1 = floorf(st.u + hx - 0.5f);
    float y0 = ceilf(st.v - hy - 0.5f), y1 = floorf(st.v + hy - 0.5f);
    const float Wm1 = float(cam.width - 1), Hm1 = float(cam.height - 1);
    x0 = fmaxf(x0, 0.f); x1 = fminf(x1, Wm1);
    y0 = fmaxf(y0, 0.f); y1 = fminf(y1, Hm1);
    if (o.flags & WS_FLAG_NO_VIEWPORT_CULL) {
        x0 = fminf(x0, Wm1); x1 = fmaxf(x1, 0.f); if (x1 < x0) x1 = x0;
        y0 = fminf(y0, Hm1); y1 = fmaxf(y1, 0.f); if (y1 < y0) y1 = y0;
    }
    if (!(x0 <= x1) || !(y0 <= y1)) return false;
    st.rect[0] = uint16_t(x0); st.rect[1] = uint16_t(x1); st.rect[2] = uint16_t(y0); st.rect[3] = uint16_t(y1);
    // key cells (tiles or bins of tiles) are powers of two in size
    const uint32_t sw = uint32_t(__builtin_ctz(uint32_t(o.cell_w()))), sh = uint32_t(__builtin_ctz(uint32_t(o.cell_h())));
    const uint32_t tx0 = st.rect[0] >> sw, tx1 = st.rect[1] >> sw;
    const uint32_t ty0 = st.rect[2] >> sh, ty1 = st.rect[3] >> sh;
    st.tiles = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
    st.visible = true;
    if (!COLOUR) return true;

    // View-dependent colour
    float dx = mx - cam.C[0], dy = my - cam.C[1], dz = mz - cam.C[2];
    st.dir_norm = sqrtf(dx * dx + dy * dy + dz * dz);
    const float idn = 1.f / st.dir_norm;
    dx *= idn; dy *= idn; dz *= idn;
    st.dir[0] = dx; st.dir[1] = dy; st.dir[2] = dz;
    float Y[16];
    sh_eval_basis(dx, dy, dz, DEG, Y);
    constexpr int K = (DEG + 1) * (DEG + 1);
    float col[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) col[ch] = fmaf(g.sh[(int64_t(k) * 3 + ch) * n + i], Y[k], col[ch]);
    }
    // a non-finite colour (non-finite SH coefficient) culls the splat as degenerate
    if (!(finitef(col[0]) && finitef(col[1]) && finitef(col[2]))) {
        st.alive = false;
        st.visible = false;
        st.tiles = 0;
        return false;
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        if (col[ch] < 0.f) { col[ch] = 0.f; st.clamp |= (1u << ch); }
        st.rgb[ch] = col[ch];
    }
    return true;
}

// ---- packed records (WS_FLAG_PACKED; Sec. 3.2's fp16 ellipse axes and RGBA8
// colour and opacity)

// The principal axes of Sigma' = [[a, b], [b, c]] (det = ac - b^2 > 0):
// sqrt(l1) v1 and sqrt(l2) v2 with l1 >= l2 its eigenvalues, v1 the unit
// eigenvector of l1 taken from (l1 - c, b) when a >= c, else (b, l1 - a)
// (the larger of the two null-space vectors of Sigma' - l1 I), v2 = v1
// turned by +90 degrees; l2 = det / l1 avoids the cancellation of mid - r.
__device__ __forceinline__ void ellipse_axes(float a, float b, float c, float det, float* ax) {
    const float hd = 0.5f * (a - c);
    const float r = sqrtf(fmaf(hd, hd, b * b));
    const float l1 = 0.5f * (a + c) + r;
    const float l2 = det / l1;
    float vx = a >= c ? l1 - c : b, vy = a >= c ? b : l1 - a;
    const float nv = sqrtf(fmaf(vx, vx, vy * vy));
    if (nv > 0.f) {
        vx /= nv;
        vy /= nv;
    } else {
        vx = 1.f;
        vy = 0.f;
    }
    const float s1 = sqrtf(l1), s2 = sqrtf(l2);
    ax[0] = s1 * vx;
    ax[1] = s1 * vy;
    ax[2] = -s2 * vy;
    ax[3] = s2 * vx;
}

// IEEE fp16 bits of x, rounded to nearest even.
__device__ __forceinline__ uint32_t half_bits(float x) {
    return uint32_t(__builtin_bit_cast(uint16_t, static_cast<_Float16>(x)));
}

// floor(255 x + 1/2) for x in [0, 1].
__device__ __forceinline__ uint32_t unorm8(float x) { return uint32_t(floorf(fmaf(x, 255.f, 0.5f))); }

}  // namespace ws
