// Plain fp64 CPU oracle for the 3D Gaussian Splatting render path.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
// reference against which the GPU library is checked.  It shares no code,
// header, table or constant with the GPU library; only the tests, the smoke
// entry point and the CPU-baseline leg of the benchmark may load it.
//
// What it computes, and where each step comes from (WebSplatter, arXiv
// 2602.03207):
//   * Gaussian model, EWA projection of the covariance and the alpha law
//     alpha = sigma * exp(-1/2 x'^T Sigma'^{-1} x')         -- Sec. 2.1, Eq. 1-2
//   * view-dependent colour c = SH(k, d), d from camera to the centre
//                                                          -- Sec. 2.1, Eq. 3
//   * front-to-back compositing C = sum c_i a_i prod_{j<i}(1-a_j)
//                                                          -- Sec. 2.1, Eq. 4
//   * culling: sigma < 1/255 dropped; AABB of the projected ellipse tested
//     against the viewport; opacity-aware cutoff radius from
//     1/255 = sigma e^{-r^2}                               -- Sec. 3.2, Sec. 3.4, Eq. 7-8
//   * (tile | depth) keys and a stable sort whose output position is
//     base_d + rank_i                                      -- Sec. 3.3.2, Eq. 5-6;
//     the <tile, splat> pair list itself is the tile-based design the paper
//     describes in Sec. 3.4.
// Readings where the paper is silent (pixel centres, low-pass dilation,
// near plane, early termination, SH sign convention, gradients at discrete
// decisions) are listed in the design notes of the repository; the code
// states each one where it is used.
//
// Threads: loops over independent items (Gaussians, tiles, pixel rows) may
// run on several host threads (OpenMP); every item is computed by the same
// code, so the results do not depend on the thread count.  The sort is
// std::stable_sort on one thread.
//
// Precision: every quantity is computed in fp64 from the caller's values.
// The only fp32 step is the depth key, which the method defines as the bits
// of the fp32 depth.
//
// Parity status: each function here is pinned by the CPU test-suite against
// something other than itself: closed forms of single Gaussians (projection,
// footprint, pixel values, gradients), brute-force compositing, culling and
// transmittance invariants, std::stable_sort / sorted(), fp64 finite
// differences, and every spherical-harmonic term against scipy's complex
// spherical harmonics converted to the real basis.  The L1 loss (in the Python
// wrapper) is pinned on hand-computed batches.  The decision-outcome
// enumeration at the end of this file is test infrastructure for comparing an
// fp32 implementation; its primary outcome is composite_pixel's result.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- interface

struct Camera {
    int32_t width, height;
    double fx, fy, cx, cy;
    double R[9];  // world -> camera rotation, row-major
    double t[3];  // p = R X + t
    double C[3];  // world-space camera centre (for the SH view direction)
};

struct Options {
    int32_t tile_w, tile_h, sh_degree, flags;
    double near_z;     // cull z <= near_z (reading of the paper's frustum cull)
    double lowpass;    // dilation added to the projected covariance diagonal
    double clamp_fov;  // projection Jacobian evaluated at x/z clamped to clamp_fov * tan(half fov)
    double alpha_min;  // splats with alpha below this are skipped (1/255)
    double alpha_max;  // alpha is clamped to this (0.99)
    double t_min;      // stop before transmittance would fall below this (1e-4)
    double bg[3];
};

constexpr int32_t FLAG_FIXED_3SIGMA = 1;   // "-RADIUS" ablation: extent 3 sigma for every splat
constexpr int32_t FLAG_NO_VIEWPORT_CULL = 2;  // "-CULL" ablation: keep splats whose AABB misses the viewport

enum Status : int8_t {
    VISIBLE = 0,
    CULL_OPACITY = 1,
    CULL_NEAR = 2,
    CULL_DEGENERATE = 3,
    CULL_VIEWPORT = 4,
};

// ------------------------------------------------------- forward-mode duals
//
// The preprocess below is written once as a template.  With T = double it is
// the forward pass; with T = Dual it also carries the derivatives of every
// output with respect to the 11 per-Gaussian geometric parameters (mean 3,
// log-scale 3, quaternion 4, opacity logit 1), so the oracle's gradient is the
// exact derivative of the oracle's own forward, branch taken.

constexpr int ND = 11;

struct Dual {
    double v = 0.0;
    double d[ND] = {};
    Dual() = default;
    Dual(double x) : v(x) {}  // NOLINT: constants promote implicitly
};

inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v); for (int i = 0; i < ND; ++i) r.d[i] = -a.d[i]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) {
    Dual r(a.v / b.v);
    for (int i = 0; i < ND; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
    return r;
}
inline Dual exp(const Dual& a) { Dual r(std::exp(a.v)); for (int i = 0; i < ND; ++i) r.d[i] = r.v * a.d[i]; return r; }
inline Dual log(const Dual& a) { Dual r(std::log(a.v)); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] / a.v; return r; }
inline Dual sqrt(const Dual& a) { Dual r(std::sqrt(a.v)); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] / (2.0 * r.v); return r; }

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
using std::exp;
using std::log;
using std::sqrt;

// ------------------------------------------------------ spherical harmonics
//
// Real spherical harmonics up to degree 3 on a unit direction (x, y, z),
// ordered (l, m) = (0,0), (1,-1), (1,0), (1,1), (2,-2) ... (3,3).
// Normalisation: the textbook orthonormal real basis.  Sign: the
// Condon-Shortley phase (-1)^m is applied, which negates the odd-|m| terms
// of the phase-free real basis.  The paper only writes c = SH(k, d) (Eq. 3);
// this is the convention of trained 3DGS scenes.

template <class T>
void sh_basis(const T& x, const T& y, const T& z, int degree, T* Y) {
    const double pi = 3.14159265358979323846;
    Y[0] = T(0.5 * std::sqrt(1.0 / pi));
    if (degree < 1) return;
    const double k1 = std::sqrt(3.0 / (4.0 * pi));
    Y[1] = T(-k1) * y;
    Y[2] = T(k1) * z;
    Y[3] = T(-k1) * x;
    if (degree < 2) return;
    const double k2a = 0.5 * std::sqrt(15.0 / pi);   // xy, yz, xz terms
    const double k2b = 0.25 * std::sqrt(5.0 / pi);   // 3z^2 - 1
    const double k2c = 0.25 * std::sqrt(15.0 / pi);  // x^2 - y^2
    Y[4] = T(k2a) * x * y;
    Y[5] = T(-k2a) * y * z;
    Y[6] = T(k2b) * (T(2.0) * z * z - x * x - y * y);
    Y[7] = T(-k2a) * x * z;
    Y[8] = T(k2c) * (x * x - y * y);
    if (degree < 3) return;
    const double k3a = 0.25 * std::sqrt(35.0 / (2.0 * pi));  // m = +-3
    const double k3b = 0.5 * std::sqrt(105.0 / pi);          // m = -2
    const double k3c = 0.25 * std::sqrt(21.0 / (2.0 * pi));  // m = +-1
    const double k3d = 0.25 * std::sqrt(7.0 / pi);           // m = 0
    const double k3e = 0.25 * std::sqrt(105.0 / pi);         // m = +2
    Y[9] = T(-k3a) * y * (T(3.0) * x * x - y * y);
    Y[10] = T(k3b) * x * y * z;
    Y[11] = T(-k3c) * y * (T(4.0) * z * z - x * x - y * y);
    Y[12] = T(k3d) * z * (T(2.0) * z * z - T(3.0) * x * x - T(3.0) * y * y);
    Y[13] = T(-k3c) * x * (T(4.0) * z * z - x * x - y * y);
    Y[14] = T(k3e) * z * (x * x - y * y);
    Y[15] = T(-k3a) * x * (x * x - T(3.0) * y * y);
}

// ------------------------------------------------------------- preprocess

template <class T>
struct Projected {
    int8_t status = CULL_DEGENERATE;
    bool valid = false;  // finite projection: passes the near-plane and degeneracy tests
    T u, v;          // projected centre, pixels
    T A, B, Cc;      // conic = inverse of the projected 2D covariance (Eq. 2)
    T cov[3];        // projected 2D covariance Sigma' (00, 01, 11) incl. dilation
    T sigma;         // peak opacity
    T rgb[3];
    double z = 0.0;  // camera-space depth
    float depth32 = 0.0f;
    uint8_t clamp_bits = 0;  // bit c: colour channel c clamped; bit 3/4: Jacobian x/y clamped
    double sh_basis_val[16] = {};  // SH basis at the view direction (for the SH gradient)
    // culling geometry
    double bound[4] = {};  // unrounded pixel-centre bounds: x_lo, x_hi, y_lo, y_hi
    int32_t pix[4] = {0, -1, 0, -1};   // inclusive pixel range x0, x1, y0, y1
    int32_t tile[4] = {0, -1, 0, -1};  // inclusive tile range
    int64_t tiles_touched = 0;
};

template <class T>
void matmul3(const T* a, const T* b, T* out) {  // out = a * b, 3x3 row-major
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            T s(0.0);
            for (int k = 0; k < 3; ++k) s = s + a[i * 3 + k] * b[k * 3 + j];
            out[i * 3 + j] = s;
        }
}

template <class T>
void transpose3(const T* a, T* out) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) out[j * 3 + i] = a[i * 3 + j];
}

// Rotation matrix of a unit quaternion (w, x, y, z): the textbook formula.
template <class T>
void quat_to_rotmat(const T* q, T* Rm) {
    const T w = q[0], x = q[1], y = q[2], z = q[3];
    const T one(1.0), two(2.0);
    Rm[0] = one - two * (y * y + z * z); Rm[1] = two * (x * y - w * z);       Rm[2] = two * (x * z + w * y);
    Rm[3] = two * (x * y + w * z);       Rm[4] = one - two * (x * x + z * z); Rm[5] = two * (y * z - w * x);
    Rm[6] = two * (x * z - w * y);       Rm[7] = two * (y * z + w * x);       Rm[8] = one - two * (x * x + y * y);
}

inline bool finite(double x) { return std::isfinite(x); }

// One Gaussian seen by one camera.  mean[3], log_scale[3], quat[4], logit are
// the geometric parameters (as T so that derivatives can ride along); sh points
// at the 3*K coefficients of this Gaussian (row k*3 + c), read at stride `shs`.
template <class T>
Projected<T> project(const T* mean, const T* log_scale, const T* quat, const T& logit,
                     const double* sh, int64_t shs, const Camera& cam, const Options& opt) {
    Projected<T> P;
    // Peak opacity; drop splats below the 8-bit quantisation step (Sec. 3.4).
    P.sigma = T(1.0) / (T(1.0) + exp(-logit));
    const double sig = val(P.sigma);

    // Camera-space centre (view-space depth, Sec. 3.1).
    T p[3];
    for (int i = 0; i < 3; ++i)
        p[i] = T(cam.R[i * 3 + 0]) * mean[0] + T(cam.R[i * 3 + 1]) * mean[1] + T(cam.R[i * 3 + 2]) * mean[2] + T(cam.t[i]);
    P.z = val(p[2]);
    P.depth32 = static_cast<float>(P.z);

    const bool finite_in = finite(val(mean[0])) && finite(val(mean[1])) && finite(val(mean[2])) &&
                           finite(val(log_scale[0])) && finite(val(log_scale[1])) && finite(val(log_scale[2])) &&
                           finite(val(quat[0])) && finite(val(quat[1])) && finite(val(quat[2])) && finite(val(quat[3])) &&
                           finite(val(logit));
    if (!finite_in) { P.status = CULL_DEGENERATE; return P; }

    // 3D covariance from rotation and scale (Sec. 2.1): Sigma = R S S^T R^T.
    T qn2 = quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3];
    if (!(val(qn2) > 0.0)) { P.status = CULL_DEGENERATE; return P; }
    T qn = sqrt(qn2);
    T qh[4] = {quat[0] / qn, quat[1] / qn, quat[2] / qn, quat[3] / qn};
    T Rq[9];
    quat_to_rotmat(qh, Rq);
    T S2[3] = {exp(T(2.0) * log_scale[0]), exp(T(2.0) * log_scale[1]), exp(T(2.0) * log_scale[2])};
    T Sigma[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            T s(0.0);
            for (int k = 0; k < 3; ++k) s = s + Rq[i * 3 + k] * S2[k] * Rq[j * 3 + k];
            Sigma[i * 3 + j] = s;
        }
    // Camera-space covariance W Sigma W^T.
    T W[9], Wt[9], tmp[9], Sc[9];
    for (int i = 0; i < 9; ++i) W[i] = T(cam.R[i]);
    transpose3(W, Wt);
    matmul3(W, Sigma, tmp);
    matmul3(tmp, Wt, Sc);

    const bool near_ok = P.z > opt.near_z;

    // Jacobian of the perspective projection at the centre, with the centre's
    // x/z and y/z clamped to clamp_fov times the half-field-of-view tangent.
    const double limx = opt.clamp_fov * (0.5 * cam.width / cam.fx);
    const double limy = opt.clamp_fov * (0.5 * cam.height / cam.fy);
    T z = p[2];
    T rx = p[0] / z, ry = p[1] / z;
    if (val(rx) > limx) { rx = T(limx); P.clamp_bits |= 8; }
    if (val(rx) < -limx) { rx = T(-limx); P.clamp_bits |= 8; }
    if (val(ry) > limy) { ry = T(limy); P.clamp_bits |= 16; }
    if (val(ry) < -limy) { ry = T(-limy); P.clamp_bits |= 16; }
    // J = [[fx/z, 0, -fx*rx/z], [0, fy/z, -fy*ry/z]]  (rx = x/z, so -fx x / z^2)
    T J0[3] = {T(cam.fx) / z, T(0.0), T(-cam.fx) * rx / z};
    T J1[3] = {T(0.0), T(cam.fy) / z, T(-cam.fy) * ry / z};
    // Sigma' = J Sc J^T + lowpass * I
    T JS0[3], JS1[3];
    for (int j = 0; j < 3; ++j) {
        JS0[j] = J0[0] * Sc[0 * 3 + j] + J0[1] * Sc[1 * 3 + j] + J0[2] * Sc[2 * 3 + j];
        JS1[j] = J1[0] * Sc[0 * 3 + j] + J1[1] * Sc[1 * 3 + j] + J1[2] * Sc[2 * 3 + j];
    }
    T a = JS0[0] * J0[0] + JS0[1] * J0[1] + JS0[2] * J0[2] + T(opt.lowpass);
    T b = JS0[0] * J1[0] + JS0[1] * J1[1] + JS0[2] * J1[2];
    T c = JS1[0] * J1[0] + JS1[1] * J1[1] + JS1[2] * J1[2] + T(opt.lowpass);
    P.cov[0] = a; P.cov[1] = b; P.cov[2] = c;
    T det = a * c - b * b;
    // Conic (A, B, C) = inverse of Sigma' (Eq. 2).
    P.A = c / det;
    P.B = -b / det;
    P.Cc = a / det;
    // Projected centre; pixel (i, j) has its centre at (i + 0.5, j + 0.5).
    P.u = T(cam.fx) * p[0] / z + T(cam.cx);
    P.v = T(cam.fy) * p[1] / z + T(cam.cy);

    // View-dependent colour (Eq. 3): d = (X - C) / |X - C|, c = max(0, SH + 0.5).
    T dir[3] = {mean[0] - T(cam.C[0]), mean[1] - T(cam.C[1]), mean[2] - T(cam.C[2])};
    T dn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    T dx = dir[0] / dn, dy = dir[1] / dn, dz = dir[2] / dn;
    const int K = (opt.sh_degree + 1) * (opt.sh_degree + 1);
    T Y[16];
    sh_basis(dx, dy, dz, opt.sh_degree, Y);
    for (int k = 0; k < K; ++k) P.sh_basis_val[k] = val(Y[k]);
    for (int ch = 0; ch < 3; ++ch) {
        T s(0.5);
        for (int k = 0; k < K; ++k) s = s + T(sh[(k * 3 + ch) * shs]) * Y[k];
        if (val(s) < 0.0) { s = T(0.0); P.clamp_bits |= uint8_t(1u << ch); }
        P.rgb[ch] = s;
    }

    // Culling, in order: opacity (Sec. 3.4), near plane, degenerate, viewport (Sec. 3.2).
    // Degenerate also covers a non-finite colour (a non-finite SH coefficient).
    const bool colour_ok = finite(val(P.rgb[0])) && finite(val(P.rgb[1])) && finite(val(P.rgb[2]));
    const bool det_ok = val(det) > 0.0 && finite(val(det)) && finite(val(P.u)) && finite(val(P.v)) && colour_ok;
    P.valid = near_ok && det_ok;
    if (!(sig >= opt.alpha_min)) { P.status = CULL_OPACITY; return P; }
    if (!near_ok) { P.status = CULL_NEAR; return P; }
    if (!det_ok) { P.status = CULL_DEGENERATE; return P; }

    // Opacity-aware extent (Sec. 3.4, Eq. 7-8): alpha = sigma e^{-m^2/2} reaches
    // alpha_min at the Mahalanobis radius m = d with d^2 = 2 ln(sigma/alpha_min).
    // The "-RADIUS" ablation uses a fixed d = 3 instead.
    const double d2 = (opt.flags & FLAG_FIXED_3SIGMA) ? 9.0 : 2.0 * std::log(sig / opt.alpha_min);
    const double hx = std::sqrt(d2 * val(a));
    const double hy = std::sqrt(d2 * val(c));
    const double uu = val(P.u), vv = val(P.v);
    // A pixel centre i + 0.5 lies in [u - hx, u + hx] iff u - hx - 0.5 <= i <= u + hx - 0.5.
    P.bound[0] = uu - hx - 0.5; P.bound[1] = uu + hx - 0.5;
    P.bound[2] = vv - hy - 0.5; P.bound[3] = vv + hy - 0.5;
    double x0 = std::ceil(P.bound[0]), x1 = std::floor(P.bound[1]);
    double y0 = std::ceil(P.bound[2]), y1 = std::floor(P.bound[3]);
    x0 = std::max(x0, 0.0); x1 = std::min(x1, double(cam.width - 1));
    y0 = std::max(y0, 0.0); y1 = std::min(y1, double(cam.height - 1));
    if (opt.flags & FLAG_NO_VIEWPORT_CULL) {
        // keep the splat: snap an empty range onto the nearest border pixel
        x0 = std::min(x0, double(cam.width - 1)); x1 = std::max(x1, 0.0); if (x1 < x0) x1 = x0;
        y0 = std::min(y0, double(cam.height - 1)); y1 = std::max(y1, 0.0); if (y1 < y0) y1 = y0;
    }
    if (!(x0 <= x1) || !(y0 <= y1)) { P.status = CULL_VIEWPORT; return P; }
    P.pix[0] = int32_t(x0); P.pix[1] = int32_t(x1); P.pix[2] = int32_t(y0); P.pix[3] = int32_t(y1);
    P.tile[0] = P.pix[0] / opt.tile_w; P.tile[1] = P.pix[1] / opt.tile_w;
    P.tile[2] = P.pix[2] / opt.tile_h; P.tile[3] = P.pix[3] / opt.tile_h;
    P.tiles_touched = int64_t(P.tile[1] - P.tile[0] + 1) * int64_t(P.tile[3] - P.tile[2] + 1);
    P.status = VISIBLE;
    return P;
}

struct GaussArrays {
    int64_t n;
    const double *means, *log_scales, *quats, *logits, *sh;  // SoA [comp][n]
};

Projected<double> project_one(const GaussArrays& g, int64_t i, const Camera& cam, const Options& opt) {
    double m[3] = {g.means[i], g.means[g.n + i], g.means[2 * g.n + i]};
    double s[3] = {g.log_scales[i], g.log_scales[g.n + i], g.log_scales[2 * g.n + i]};
    double q[4] = {g.quats[i], g.quats[g.n + i], g.quats[2 * g.n + i], g.quats[3 * g.n + i]};
    return project<double>(m, s, q, g.logits[i], g.sh + i, g.n, cam, opt);
}

Projected<Dual> project_dual(const GaussArrays& g, int64_t i, const Camera& cam, const Options& opt) {
    Dual m[3], s[3], q[4], o;
    for (int k = 0; k < 3; ++k) { m[k] = Dual(g.means[k * g.n + i]); m[k].d[k] = 1.0; }
    for (int k = 0; k < 3; ++k) { s[k] = Dual(g.log_scales[k * g.n + i]); s[k].d[3 + k] = 1.0; }
    for (int k = 0; k < 4; ++k) { q[k] = Dual(g.quats[k * g.n + i]); q[k].d[6 + k] = 1.0; }
    o = Dual(g.logits[i]); o.d[10] = 1.0;
    return project<Dual>(m, s, q, o, g.sh + i, g.n, cam, opt);
}

// ---------------------------------------------------------- compositing
//
// Front-to-back alpha compositing of one pixel (Eq. 2 and Eq. 4), with the
// readings: alpha = min(alpha_max, sigma exp(power)); a splat with
// alpha < alpha_min is skipped; if the transmittance after a splat would fall
// below t_min the pixel stops *before* compositing that splat.

struct PixelSplat {  // what compositing needs of one projected splat
    double u, v, A, B, C, sigma, rgb[3];
    int32_t x0, x1, y0, y1;  // inclusive pixel rectangle (the culling AABB)
};

struct Contrib {
    int64_t id;
    double alpha, T, dx, dy, G;  // G = exp(power)
    bool clamped;
};

struct PixelResult {
    double rgb[3];
    double T;
    int64_t n_eval;          // list entries visited (including skipped ones) before stopping
    int64_t n_contrib;
    double alpha_margin;     // min |ln(alpha_raw / alpha_min)| over visited entries
    double t_margin;         // min |ln(T' / t_min)| over the transmittance tests
    uint64_t hash;           // hash of the per-entry decisions
};

inline uint64_t mix(uint64_t h, uint64_t x) {
    h ^= x + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
    return h;
}

// A splat is evaluated at a pixel only if the pixel lies in the splat's
// pixel rectangle.  With the opacity-aware extent this test never removes a
// splat whose alpha reaches alpha_min (Sec. 3.4), so the result equals
// brute-force compositing; under the fixed-3-sigma ablation it clips.
template <class GetSplat>
PixelResult composite_pixel(int32_t px, int32_t py, const int64_t* ids, int64_t count, GetSplat get,
                            const Options& opt, std::vector<Contrib>* contribs) {
    const double pcx = px + 0.5, pcy = py + 0.5;
    PixelResult r{};
    r.T = 1.0;
    r.alpha_margin = INFINITY;
    r.t_margin = INFINITY;
    r.hash = 1469598103934665603ULL;
    double T = 1.0;
    for (int64_t j = 0; j < count; ++j) {
        const PixelSplat& s = get(ids[j]);
        if (px < s.x0 || px > s.x1 || py < s.y0 || py > s.y1) continue;
        r.n_eval += 1;
        const double dx = s.u - pcx, dy = s.v - pcy;
        const double power = -0.5 * (s.A * dx * dx + s.C * dy * dy) - s.B * dx * dy;
        const double G = std::exp(power);
        const double alpha_raw = s.sigma * G;
        const double alpha = std::min(opt.alpha_max, alpha_raw);
        if (s.sigma > 0.0)
            r.alpha_margin = std::min(r.alpha_margin, std::fabs(std::log(s.sigma / opt.alpha_min) + power));
        if (alpha < opt.alpha_min) { r.hash = mix(r.hash, uint64_t(ids[j]) * 4 + 0); continue; }
        const double Tn = T * (1.0 - alpha);
        r.t_margin = std::min(r.t_margin, std::fabs(std::log(Tn / opt.t_min)));
        if (Tn < opt.t_min) { r.hash = mix(r.hash, uint64_t(ids[j]) * 4 + 3); break; }
        const bool clamped = alpha_raw > opt.alpha_max;
        r.hash = mix(r.hash, uint64_t(ids[j]) * 4 + (clamped ? 2 : 1));
        for (int ch = 0; ch < 3; ++ch) r.rgb[ch] += s.rgb[ch] * alpha * T;
        if (contribs) contribs->push_back(Contrib{ids[j], alpha, T, dx, dy, G, clamped});
        T = Tn;
        r.n_contrib += 1;
    }
    r.T = T;
    for (int ch = 0; ch < 3; ++ch) r.rgb[ch] += T * opt.bg[ch];
    return r;
}

// Reverse mode of composite_pixel for one pixel: adds dL/d(u, v, A, B, C, sigma, r, g, b)
// of every contributing splat into grad[id*9 + k], given dL/dC for the pixel.
void composite_pixel_adjoint(const std::vector<Contrib>& cs, double T_final,
                             const double* dLdC, const std::vector<PixelSplat>& splats,
                             const Options& opt, double* grad) {
    // R_k = sum_{i>k} c_i a_i T_i + bg T_final  (suffix of the composite)
    double Rsum[3] = {opt.bg[0] * T_final, opt.bg[1] * T_final, opt.bg[2] * T_final};
    for (int64_t k = int64_t(cs.size()) - 1; k >= 0; --k) {
        const Contrib& c = cs[size_t(k)];
        const PixelSplat& s = splats[size_t(c.id)];
        double* g = grad + c.id * 9;
        // dC/dc_k = a_k T_k ; dC/da_k = c_k T_k - R_k / (1 - a_k)
        double dL_dalpha = 0.0;
        for (int ch = 0; ch < 3; ++ch) {
            g[6 + ch] += dLdC[ch] * c.alpha * c.T;
            dL_dalpha += dLdC[ch] * (s.rgb[ch] * c.T - Rsum[ch] / (1.0 - c.alpha));
        }
        for (int ch = 0; ch < 3; ++ch) Rsum[ch] += s.rgb[ch] * c.alpha * c.T;
        if (c.clamped) continue;  // alpha = alpha_max: no dependence on sigma or power
        // alpha = sigma G, G = exp(power), power = -1/2 (A dx^2 + C dy^2) - B dx dy, dx = u - pcx
        g[5] += dL_dalpha * c.G;
        const double dL_dpower = dL_dalpha * s.sigma * c.G;
        g[0] += dL_dpower * (-(s.A * c.dx + s.B * c.dy));
        g[1] += dL_dpower * (-(s.C * c.dy + s.B * c.dx));
        g[2] += dL_dpower * (-0.5 * c.dx * c.dx);
        g[3] += dL_dpower * (-(c.dx * c.dy));
        g[4] += dL_dpower * (-0.5 * c.dy * c.dy);
    }
}

// Projected splat of every Gaussian for a view, plus decision records.
// Loops over independent items (Gaussians, tiles, pixel rows) carry OpenMP
// work-sharing pragmas: with an OpenMP build and more than one thread they run
// on several host cores and give the same bits, each item being computed by
// the same code whatever thread runs it; without OpenMP they are plain loops.
void project_all(const GaussArrays& g, const Camera& cam, const Options& opt, std::vector<Projected<double>>& out) {
    out.resize(size_t(g.n));
#pragma omp parallel for schedule(static, 4096)
    for (int64_t i = 0; i < g.n; ++i) out[size_t(i)] = project_one(g, i, cam, opt);
}

std::vector<PixelSplat> splats_of(const std::vector<Projected<double>>& P) {
    std::vector<PixelSplat> s(P.size());
    for (size_t i = 0; i < P.size(); ++i) {
        const auto& p = P[i];
        s[i] = PixelSplat{p.u, p.v, p.A, p.B, p.Cc, p.sigma, {p.rgb[0], p.rgb[1], p.rgb[2]},
                          p.pix[0], p.pix[1], p.pix[2], p.pix[3]};
    }
    return s;
}

// Pair emission (tile-major keys): for each visible Gaussian in id order, its
// tiles in row-major order; key = (tile_offset + ty*tiles_x + tx) << 32 | bits(fp32 depth).
int64_t emit_pairs(const std::vector<Projected<double>>& P, int64_t tile_offset, int32_t tiles_x,
                   uint64_t* keys, uint32_t* vals, int64_t capacity) {
    int64_t m = 0;
    for (size_t i = 0; i < P.size(); ++i) {
        const auto& p = P[i];
        if (p.status != VISIBLE) continue;
        uint32_t dbits;
        std::memcpy(&dbits, &p.depth32, 4);
        for (int32_t ty = p.tile[2]; ty <= p.tile[3]; ++ty)
            for (int32_t tx = p.tile[0]; tx <= p.tile[1]; ++tx) {
                if (m < capacity) {
                    const uint64_t tile = uint64_t(tile_offset + int64_t(ty) * tiles_x + tx);
                    keys[m] = (tile << 32) | dbits;
                    vals[m] = uint32_t(i);
                }
                ++m;
            }
    }
    return m;
}

// Stable sort of (key, value) pairs on key bits [begin_bit, end_bit): the
// plain definition of the LSD radix sort's result (Sec. 3.3.2: equal digits
// keep their input order).
void stable_sort_pairs(int64_t n, uint64_t* keys, uint32_t* vals, int begin_bit, int end_bit) {
    const uint64_t mask = (end_bit - begin_bit >= 64) ? ~0ULL : (((1ULL << (end_bit - begin_bit)) - 1ULL) << begin_bit);
    std::vector<int64_t> idx(static_cast<size_t>(n));
    std::iota(idx.begin(), idx.end(), int64_t(0));
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return (keys[a] & mask) < (keys[b] & mask); });
    std::vector<uint64_t> k2(static_cast<size_t>(n));
    std::vector<uint32_t> v2(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) { k2[size_t(i)] = keys[idx[size_t(i)]]; v2[size_t(i)] = vals[idx[size_t(i)]]; }
    std::copy(k2.begin(), k2.end(), keys);
    std::copy(v2.begin(), v2.end(), vals);
}

// ------------------------------------------- decisions within fp32 reach
//
// Test infrastructure for parity with an fp32 implementation.  The GPU
// evaluates the same rule from fp32-rounded splat records in fp32, so each of
// its discrete decisions (alpha >= alpha_min, T' < t_min) may differ from the
// fp64 one wherever the fp64 value lies within the fp32 error of the
// threshold, and each choice there is a correct result of the rule (several
// correct results: reading A25).  For one pixel this enumerates, depth first,
// the composites of every combination of such decisions.
//
// Error bound of ln(alpha) as the fp32 path computes it (ln units):
//   the centre rounded to fp32 (at most 2^-23 |u| per coordinate) times the
//   gradient of the exponent in the centre, plus 2^-18 (cond + 1)(|power| + 1)
//   for the conic's rounding and the evaluation (cond = the conic's condition
//   number), plus 2^-18 (|ln sigma| + 1).
// Error bound of ln(T): the sum over the composited splats of
// alpha / (1 - alpha) times their ln(alpha) bound, plus 2^-22 per step.
struct SplatError {  // the per-splat parts of the bound
    double eu, ev;      // 2^-23 (|u| + 1), 2^-23 (|v| + 1)
    double cond1;       // 2^-18 (cond + 1)
    double ls;          // 2^-18 (|ln sigma| + 1)
    double ln_sigma_rel;  // ln(sigma / alpha_min)
};

SplatError splat_error(const PixelSplat& s, const Options& opt) {
    SplatError e;
    e.eu = std::ldexp(std::fabs(s.u) + 1.0, -23);
    e.ev = std::ldexp(std::fabs(s.v) + 1.0, -23);
    const double tr = s.A + s.C, det = s.A * s.C - s.B * s.B;
    const double disc = std::sqrt(std::max(tr * tr - 4.0 * det, 0.0));
    const double lmin = 0.5 * (tr - disc), lmax = 0.5 * (tr + disc);
    e.cond1 = std::ldexp((lmin > 0.0 ? lmax / lmin : 1e30) + 1.0, -18);
    e.ls = s.sigma > 0.0 ? std::ldexp(std::fabs(std::log(s.sigma)) + 1.0, -18) : 0.0;
    e.ln_sigma_rel = s.sigma > 0.0 ? std::log(s.sigma / opt.alpha_min) : -INFINITY;
    return e;
}

double alpha_log_error(const PixelSplat& s, const SplatError& e, double dx, double dy, double power) {
    const double gu = std::fabs(s.A * dx + s.B * dy), gv = std::fabs(s.B * dx + s.C * dy);
    return gu * e.eu + gv * e.ev + e.cond1 * (std::fabs(power) + 1.0) + e.ls;
}

struct OutcomeSearch {
    const std::vector<PixelSplat>* S;
    const std::vector<SplatError>* E;
    const int64_t* ids;
    int64_t count;
    const Options* opt;
    int32_t px, py;
    double pcx, pcy;
    size_t max_out;
    std::vector<double> out;  // 3 per outcome
    bool capped = false;
    bool uncertain = false;
    double first_T = 0.0;  // transmittance at the first decision within reach

    void record(const double* C, double T) {
        double v[3];
        for (int ch = 0; ch < 3; ++ch) v[ch] = C[ch] + T * opt->bg[ch];
        for (size_t k = 0; k < out.size(); k += 3)
            if (out[k] == v[0] && out[k + 1] == v[1] && out[k + 2] == v[2]) return;
        if (out.size() / 3 >= max_out) { capped = true; return; }
        out.insert(out.end(), v, v + 3);
    }
    void mark(double T) {
        if (!uncertain) first_T = T;
        uncertain = true;
    }

    // continue the pixel from list entry j with transmittance T, colour C and
    // the error bound lnT_err of ln T
    void run(int64_t j, double T, const double* Cin, double lnT_err) {
        if (capped) return;
        double C[3] = {Cin[0], Cin[1], Cin[2]};
        for (; j < count; ++j) {
            const PixelSplat& s = (*S)[size_t(ids[j])];
            const bool in_rect = !(px < s.x0 || px > s.x1 || py < s.y0 || py > s.y1);
            const double dx = s.u - pcx, dy = s.v - pcy;
            const double power = -0.5 * (s.A * dx * dx + s.C * dy * dy) - s.B * dx * dy;
            const SplatError& se = (*E)[size_t(ids[j])];
            const double ea = s.sigma > 0.0 ? alpha_log_error(s, se, dx, dy, power) : 0.0;
            const double la = se.ln_sigma_rel + power;
            // Outside the rectangle the rule never composites (reading A27);
            // an fp32 evaluation that tests alpha alone takes the splat there
            // only where its alpha test is within reach, the one case the
            // enumeration below follows.
            if (!in_rect && !(std::fabs(la) <= ea)) continue;
            const double alpha_raw = s.sigma * std::exp(power);
            const double alpha = std::min(opt->alpha_max, alpha_raw);
            const bool take_here = in_rect && alpha >= opt->alpha_min;
            if (std::fabs(la) <= ea && alpha_raw > 0.0) {  // the alpha test within reach: both choices valid
                mark(T);
                if (take_here) {
                    run(j + 1, T, C, lnT_err);  // the other choice: skip j
                } else if (take(j, T, C, lnT_err, alpha, ea)) {  // the other choice: take j
                    double Cn[3];
                    for (int ch = 0; ch < 3; ++ch) Cn[ch] = C[ch] + s.rgb[ch] * alpha * T;
                    run(j + 1, T * (1.0 - alpha), Cn, lnT_err + alpha / (1.0 - alpha) * ea + std::ldexp(1.0, -22));
                }
            }
            if (!take_here) continue;
            if (!take(j, T, C, lnT_err, alpha, ea)) return;  // stopped (its outcomes are recorded)
            for (int ch = 0; ch < 3; ++ch) C[ch] += s.rgb[ch] * alpha * T;
            lnT_err += alpha / (1.0 - alpha) * ea + std::ldexp(1.0, -22);
            T *= 1.0 - alpha;
        }
        record(C, T);
    }

    // Splat j is taken (alpha >= alpha_min).  Applies the transmittance test:
    // returns true if the pixel continues past j with this splat composited
    // (the caller updates T and C), false when every continuation has been
    // handled here.
    bool take(int64_t j, double T, const double* C, double lnT_err, double alpha, double ea) {
        const PixelSplat& s = (*S)[size_t(ids[j])];
        const double Tn = T * (1.0 - alpha);
        const double et = lnT_err + alpha / (1.0 - alpha) * ea + std::ldexp(1.0, -21);
        const double lt = std::log(Tn / opt->t_min);
        if (std::fabs(lt) <= et) {  // the stop test within reach: both valid
            mark(T);
            record(C, T);  // stop before j
            double Cn[3];
            for (int ch = 0; ch < 3; ++ch) Cn[ch] = C[ch] + s.rgb[ch] * alpha * T;
            run(j + 1, Tn, Cn, lnT_err + alpha / (1.0 - alpha) * ea + std::ldexp(1.0, -22));
            return false;
        }
        if (Tn < opt->t_min) {
            record(C, T);
            return false;
        }
        return true;
    }
};

}  // namespace

// ======================================================================
// C interface (called through ctypes from the Python test helpers)
// ======================================================================

extern "C" {

struct orc_projected {  // output arrays, each of length n (or [k][n])
    int8_t* status;
    double* mean2d;  // [2][n]
    double* conic;   // [3][n]
    double* cov2d;   // [3][n]
    double* z;
    float* depth32;
    double* opacity;
    double* rgb;     // [3][n]
    int32_t* pix_rect;   // [4][n]  x0, x1, y0, y1 inclusive
    int32_t* tile_rect;  // [4][n]
    int64_t* tiles_touched;
    uint8_t* clamp_bits;
    double* bounds;  // [4][n] unrounded bounds
};

// Projection, colour and culling of every Gaussian for one camera.
int orc_preprocess(int64_t n, const double* means, const double* log_scales, const double* quats,
                   const double* logits, const double* sh, const Camera* cam, const Options* opt,
                   orc_projected* out) {
    GaussArrays g{n, means, log_scales, quats, logits, sh};
    for (int64_t i = 0; i < n; ++i) {
        Projected<double> p = project_one(g, i, *cam, *opt);
        out->status[i] = p.status;
        out->mean2d[i] = p.u; out->mean2d[n + i] = p.v;
        out->conic[i] = p.A; out->conic[n + i] = p.B; out->conic[2 * n + i] = p.Cc;
        for (int k = 0; k < 3; ++k) out->cov2d[k * n + i] = p.cov[k];
        out->z[i] = p.z;
        out->depth32[i] = p.depth32;
        out->opacity[i] = p.sigma;
        for (int k = 0; k < 3; ++k) out->rgb[k * n + i] = p.rgb[k];
        for (int k = 0; k < 4; ++k) {
            out->pix_rect[k * n + i] = p.pix[k];
            out->tile_rect[k * n + i] = p.tile[k];
            out->bounds[k * n + i] = p.bound[k];
        }
        out->tiles_touched[i] = p.tiles_touched;
        out->clamp_bits[i] = p.clamp_bits;
    }
    return 0;
}

// Key emission for one view from preprocess outputs; returns the pair count
// (pairs beyond `capacity` are counted but not written).
int64_t orc_emit(int64_t n, const Camera* cam, const Options* opt, const double* means, const double* log_scales,
                 const double* quats, const double* logits, const double* sh, int64_t tile_offset,
                 uint64_t* keys, uint32_t* vals, int64_t capacity) {
    GaussArrays g{n, means, log_scales, quats, logits, sh};
    std::vector<Projected<double>> P;
    project_all(g, *cam, *opt, P);
    const int32_t tiles_x = (cam->width + opt->tile_w - 1) / opt->tile_w;
    return emit_pairs(P, tile_offset, tiles_x, keys, vals, capacity);
}

void orc_stable_sort(int64_t n, uint64_t* keys, uint32_t* vals, int32_t begin_bit, int32_t end_bit) {
    stable_sort_pairs(n, keys, vals, begin_bit, end_bit);
}

// Per-tile [start, end) ranges of a tile-sorted key list; tiles with no pair get [0, 0).
void orc_tile_ranges(int64_t n, const uint64_t* keys, int64_t n_tiles, int64_t* ranges) {
    for (int64_t t = 0; t < 2 * n_tiles; ++t) ranges[t] = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t tile = int64_t(keys[i] >> 32);
        if (i == 0 || int64_t(keys[i - 1] >> 32) != tile) ranges[2 * tile] = i;
        if (i == n - 1 || int64_t(keys[i + 1] >> 32) != tile) ranges[2 * tile + 1] = i + 1;
    }
}

struct orc_image {  // per-view outputs of compositing; any pointer may be null
    double* rgb;            // [3][H][W]
    double* T;              // [H][W]
    int64_t* n_eval;        // [H][W]
    int64_t* n_contrib;     // [H][W]
    double* alpha_margin;   // [H][W]
    double* t_margin;       // [H][W]
    uint64_t* hash;         // [H][W]
};

// Tiled compositing from given projected splats (fp64 arrays, e.g. the
// oracle's own or fp32 values widened) and a tile-sorted pair list.  Only the
// pixels with mask != 0 are composited (mask may be null = all).
int orc_composite(int64_t n, const double* mean2d, const double* conic, const double* opacity, const double* rgb,
                  const int32_t* pix_rect, const Camera* cam, const Options* opt, int64_t n_pairs,
                  const uint32_t* vals, const int64_t* ranges, int64_t tile_offset, const uint8_t* mask,
                  orc_image* out) {
    std::vector<PixelSplat> S(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i)
        S[size_t(i)] = PixelSplat{mean2d[i], mean2d[n + i], conic[i], conic[n + i], conic[2 * n + i], opacity[i],
                                  {rgb[i], rgb[n + i], rgb[2 * n + i]},
                                  pix_rect[i], pix_rect[n + i], pix_rect[2 * n + i], pix_rect[3 * n + i]};
    const int32_t W = cam->width, H = cam->height;
    const int32_t tx_n = (W + opt->tile_w - 1) / opt->tile_w, ty_n = (H + opt->tile_h - 1) / opt->tile_h;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < int64_t(tx_n) * ty_n; ++t) {
        std::vector<int64_t> ids;
        const int32_t ty = int32_t(t / tx_n), tx = int32_t(t % tx_n);
        const int64_t tile = tile_offset + int64_t(ty) * tx_n + tx;
        const int64_t s = ranges[2 * tile], e = ranges[2 * tile + 1];
        ids.resize(size_t(e - s));
        for (int64_t j = s; j < e; ++j) ids[size_t(j - s)] = vals[j];
        for (int32_t py = ty * opt->tile_h; py < std::min(H, (ty + 1) * opt->tile_h); ++py)
            for (int32_t px = tx * opt->tile_w; px < std::min(W, (tx + 1) * opt->tile_w); ++px) {
                const int64_t pix = int64_t(py) * W + px;
                if (mask && !mask[pix]) continue;
                PixelResult r = composite_pixel(px, py, ids.data(), int64_t(ids.size()),
                                                [&](int64_t id) -> const PixelSplat& { return S[size_t(id)]; },
                                                *opt, nullptr);
                if (out->rgb) for (int ch = 0; ch < 3; ++ch) out->rgb[int64_t(ch) * H * W + pix] = r.rgb[ch];
                if (out->T) out->T[pix] = r.T;
                if (out->n_eval) out->n_eval[pix] = r.n_eval;
                if (out->n_contrib) out->n_contrib[pix] = r.n_contrib;
                if (out->alpha_margin) out->alpha_margin[pix] = r.alpha_margin;
                if (out->t_margin) out->t_margin[pix] = r.t_margin;
                if (out->hash) out->hash[pix] = r.hash;
            }
    }
    (void)n_pairs;
    return 0;
}

// Brute-force compositing: every Gaussian with a valid projection (passes the
// near-plane and degeneracy tests), ordered by (fp32 depth bits, id), every
// pixel (with mask != 0; mask may be null).  No opacity, AABB, viewport or tile
// culling is applied: this is the plain definition that the culled tiled
// pipeline must reproduce.
int orc_render_brute(int64_t n, const double* means, const double* log_scales, const double* quats,
                     const double* logits, const double* sh, const Camera* cam, const Options* opt,
                     const uint8_t* mask, orc_image* out) {
    GaussArrays g{n, means, log_scales, quats, logits, sh};
    std::vector<Projected<double>> P;
    project_all(g, *cam, *opt, P);
    std::vector<int64_t> ids;
    for (int64_t i = 0; i < n; ++i) {
        if (P[size_t(i)].valid) ids.push_back(i);
    }
    std::stable_sort(ids.begin(), ids.end(), [&](int64_t a, int64_t b) {
        uint32_t da, db;
        std::memcpy(&da, &P[size_t(a)].depth32, 4);
        std::memcpy(&db, &P[size_t(b)].depth32, 4);
        return da < db;
    });
    std::vector<PixelSplat> S = splats_of(P);
    const int32_t W = cam->width, H = cam->height;
    for (auto& s : S) { s.x0 = 0; s.x1 = W - 1; s.y0 = 0; s.y1 = H - 1; }  // no rectangle test
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t py = 0; py < H; ++py)
        for (int32_t px = 0; px < W; ++px) {
            const int64_t pix = int64_t(py) * W + px;
            if (mask && !mask[pix]) continue;
            PixelResult r = composite_pixel(px, py, ids.data(), int64_t(ids.size()),
                                            [&](int64_t id) -> const PixelSplat& { return S[size_t(id)]; }, *opt, nullptr);
            if (out->rgb) for (int ch = 0; ch < 3; ++ch) out->rgb[int64_t(ch) * H * W + pix] = r.rgb[ch];
            if (out->T) out->T[pix] = r.T;
            if (out->n_eval) out->n_eval[pix] = r.n_eval;
            if (out->n_contrib) out->n_contrib[pix] = r.n_contrib;
            if (out->alpha_margin) out->alpha_margin[pix] = r.alpha_margin;
            if (out->t_margin) out->t_margin[pix] = r.t_margin;
            if (out->hash) out->hash[pix] = r.hash;
        }
    return 0;
}

// Full forward of one view (preprocess, emission, stable sort, ranges,
// compositing) followed by its reverse mode, given dL/dimage [3][H][W].
// Adds (does not overwrite) the parameter gradients into the g_* arrays and,
// if splat_grad is non-null, writes dL/d(u, v, A, B, C, sigma, r, g, b) per
// Gaussian into splat_grad[n][9].  Returns a hash of every discrete decision
// (culls, clamps, per-pixel skip/contribute/stop) so that finite-difference
// probes can be restricted to a fixed branch.
uint64_t orc_forward_backward(int64_t n, const double* means, const double* log_scales, const double* quats,
                              const double* logits, const double* sh, const Camera* cam, const Options* opt,
                              const double* dL_dimage, double* image_out, double* g_means, double* g_log_scales,
                              double* g_quats, double* g_logits, double* g_sh, double* splat_grad) {
    GaussArrays g{n, means, log_scales, quats, logits, sh};
    std::vector<Projected<double>> P;
    project_all(g, *cam, *opt, P);
    uint64_t h = 1469598103934665603ULL;
    for (int64_t i = 0; i < n; ++i) {
        const auto& p = P[size_t(i)];
        h = mix(h, uint64_t(p.status) | (uint64_t(p.clamp_bits) << 8));
        if (p.status == VISIBLE)
            for (int k = 0; k < 4; ++k) h = mix(h, uint64_t(uint32_t(p.tile[k])));
    }
    const int32_t tiles_x = (cam->width + opt->tile_w - 1) / opt->tile_w;
    const int32_t tiles_y = (cam->height + opt->tile_h - 1) / opt->tile_h;
    int64_t m = 0;
    for (const auto& p : P) if (p.status == VISIBLE) m += p.tiles_touched;
    std::vector<uint64_t> keys(static_cast<size_t>(m));
    std::vector<uint32_t> vals(static_cast<size_t>(m));
    emit_pairs(P, 0, tiles_x, keys.data(), vals.data(), m);
    stable_sort_pairs(m, keys.data(), vals.data(), 0, 64);
    std::vector<int64_t> ranges(size_t(2) * tiles_x * tiles_y);
    orc_tile_ranges(m, keys.data(), int64_t(tiles_x) * tiles_y, ranges.data());
    std::vector<PixelSplat> S = splats_of(P);
    std::vector<double> sg(size_t(n) * 9, 0.0);
    std::vector<int64_t> ids;
    std::vector<Contrib> cs;
    const int32_t W = cam->width, H = cam->height;
    for (int32_t ty = 0; ty < tiles_y; ++ty)
        for (int32_t tx = 0; tx < tiles_x; ++tx) {
            const int64_t tile = int64_t(ty) * tiles_x + tx;
            const int64_t s = ranges[size_t(2 * tile)], e = ranges[size_t(2 * tile + 1)];
            ids.resize(size_t(e - s));
            for (int64_t j = s; j < e; ++j) ids[size_t(j - s)] = vals[size_t(j)];
            for (int32_t py = ty * opt->tile_h; py < std::min(H, (ty + 1) * opt->tile_h); ++py)
                for (int32_t px = tx * opt->tile_w; px < std::min(W, (tx + 1) * opt->tile_w); ++px) {
                    const int64_t pix = int64_t(py) * W + px;
                    cs.clear();
                    PixelResult r = composite_pixel(px, py, ids.data(), int64_t(ids.size()),
                                                    [&](int64_t id) -> const PixelSplat& { return S[size_t(id)]; },
                                                    *opt, &cs);
                    h = mix(h, r.hash);
                    if (image_out) for (int ch = 0; ch < 3; ++ch) image_out[int64_t(ch) * H * W + pix] = r.rgb[ch];
                    if (dL_dimage) {
                        double dLdC[3] = {dL_dimage[pix], dL_dimage[int64_t(H) * W + pix], dL_dimage[2 * int64_t(H) * W + pix]};
                        composite_pixel_adjoint(cs, r.T, dLdC, S, *opt, sg.data());
                    }
                }
        }
    if (splat_grad) std::copy(sg.begin(), sg.end(), splat_grad);
    if (!dL_dimage) return h;
    // Preprocess adjoint: chain dL/d(u, v, A, B, C, sigma, rgb) to the parameters
    // through the exact forward-mode derivatives of project().
    const int K = (opt->sh_degree + 1) * (opt->sh_degree + 1);
    for (int64_t i = 0; i < n; ++i) {
        if (P[size_t(i)].status != VISIBLE) continue;  // culled: no contribution, zero gradient
        const double* gi = &sg[size_t(i) * 9];
        bool any = false;
        for (int k = 0; k < 9; ++k) any = any || gi[k] != 0.0;
        if (!any) continue;
        Projected<Dual> D = project_dual(g, i, *cam, *opt);
        const Dual* outs[9] = {&D.u, &D.v, &D.A, &D.B, &D.Cc, &D.sigma, &D.rgb[0], &D.rgb[1], &D.rgb[2]};
        double gp[ND] = {};
        for (int o = 0; o < 9; ++o)
            for (int k = 0; k < ND; ++k) gp[k] += gi[o] * outs[o]->d[k];
        for (int k = 0; k < 3; ++k) g_means[k * n + i] += gp[k];
        for (int k = 0; k < 3; ++k) g_log_scales[k * n + i] += gp[3 + k];
        for (int k = 0; k < 4; ++k) g_quats[k * n + i] += gp[6 + k];
        g_logits[i] += gp[10];
        // colour is linear in the SH coefficients: dc/dk_{k,ch} = Y_k(d) unless clamped
        for (int ch = 0; ch < 3; ++ch) {
            if (D.clamp_bits & (1u << ch)) continue;
            for (int k = 0; k < K; ++k) g_sh[(int64_t(k) * 3 + ch) * n + i] += gi[6 + ch] * D.sh_basis_val[k];
        }
    }
    return h;
}

// Pixels whose compositing takes a decision within fp32 reach of its
// threshold, with every composite the combinations of those decisions give
// (tiled lists as in orc_composite; pixels with mask != 0).  Writes, for up to
// cap such pixels, pix[k] (flat pixel index), n_out[k] (outcomes, at most
// max_out; 0 when the enumeration was cut at max_out), out_rgb[k][max_out][3]
// and bound[k] = the transmittance at the pixel's first such decision times
// the largest colour of its list (everything composited from there on weighs
// at most that transmittance).  Returns the number of such pixels, which may
// exceed cap (then only the first cap are written).
int64_t orc_composite_outcomes(int64_t n, const double* mean2d, const double* conic, const double* opacity,
                               const double* rgb, const int32_t* pix_rect, const Camera* cam, const Options* opt,
                               const uint32_t* vals, const int64_t* ranges, int64_t tile_offset,
                               const uint8_t* mask, int32_t max_out, int64_t cap, int64_t* pix, int32_t* n_out,
                               double* out_rgb, double* bound) {
    std::vector<PixelSplat> S(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i)
        S[size_t(i)] = PixelSplat{mean2d[i], mean2d[n + i], conic[i], conic[n + i], conic[2 * n + i], opacity[i],
                                  {rgb[i], rgb[n + i], rgb[2 * n + i]},
                                  pix_rect[i], pix_rect[n + i], pix_rect[2 * n + i], pix_rect[3 * n + i]};
    std::vector<SplatError> E(S.size());
    for (size_t i = 0; i < S.size(); ++i) E[i] = splat_error(S[i], *opt);
    const int32_t W = cam->width, H = cam->height;
    const int32_t tx_n = (W + opt->tile_w - 1) / opt->tile_w, ty_n = (H + opt->tile_h - 1) / opt->tile_h;
    struct Found {
        int64_t pix;
        int32_t n_out;
        double bound;
        std::vector<double> rgb;
    };
    const int64_t n_tiles = int64_t(tx_n) * ty_n;
    std::vector<std::vector<Found>> per_tile(static_cast<size_t>(n_tiles));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < n_tiles; ++t) {
        std::vector<int64_t> ids;
        const int32_t ty = int32_t(t / tx_n), tx = int32_t(t % tx_n);
        const int64_t tile = tile_offset + int64_t(ty) * tx_n + tx;
        const int64_t s0 = ranges[2 * tile], e0 = ranges[2 * tile + 1];
        ids.resize(size_t(e0 - s0));
        double maxc = std::max({std::fabs(opt->bg[0]), std::fabs(opt->bg[1]), std::fabs(opt->bg[2])});
        for (int64_t j = s0; j < e0; ++j) {
            ids[size_t(j - s0)] = vals[j];
            for (int ch = 0; ch < 3; ++ch) maxc = std::max(maxc, std::fabs(S[vals[j]].rgb[ch]));
        }
        for (int32_t py = ty * opt->tile_h; py < std::min(H, (ty + 1) * opt->tile_h); ++py)
            for (int32_t px = tx * opt->tile_w; px < std::min(W, (tx + 1) * opt->tile_w); ++px) {
                const int64_t p = int64_t(py) * W + px;
                if (mask && !mask[p]) continue;
                OutcomeSearch o;
                o.S = &S;
                o.E = &E;
                o.ids = ids.data();
                o.count = int64_t(ids.size());
                o.opt = opt;
                o.px = px;
                o.py = py;
                o.pcx = px + 0.5;
                o.pcy = py + 0.5;
                o.max_out = size_t(std::max(max_out, 1));
                const double C0[3] = {0.0, 0.0, 0.0};
                o.run(0, 1.0, C0, 0.0);
                if (!o.uncertain) continue;
                per_tile[size_t(t)].push_back(
                    Found{p, o.capped ? 0 : int32_t(o.out.size() / 3), o.first_T * maxc, o.out});
            }
    }
    // in tile order, as a single-threaded run lists them
    int64_t found = 0;
    for (const auto& list : per_tile)
        for (const Found& f : list) {
            if (found < cap) {
                pix[found] = f.pix;
                n_out[found] = f.n_out;
                for (size_t q = 0; q < f.rgb.size(); ++q) out_rgb[size_t(found) * size_t(max_out) * 3 + q] = f.rgb[q];
                bound[found] = f.bound;
            }
            ++found;
        }
    return found;
}

// Threads of the OpenMP work-sharing loops (1 without OpenMP).
#ifdef _OPENMP
void orc_set_threads(int32_t k) { omp_set_num_threads(k > 0 ? k : 1); }
int32_t orc_max_threads(void) { return omp_get_max_threads(); }
#else
void orc_set_threads(int32_t k) { (void)k; }
int32_t orc_max_threads(void) { return 1; }
#endif

// Building blocks exposed for the pins.
void orc_sh_basis(const double* dir, int32_t degree, double* out) {
    for (int k = 0; k < 16; ++k) out[k] = 0.0;
    sh_basis<double>(dir[0], dir[1], dir[2], degree, out);
}

void orc_quat_to_rotmat(const double* q, double* out) {
    const double nq = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double qh[4] = {q[0] / nq, q[1] / nq, q[2] / nq, q[3] / nq};
    quat_to_rotmat<double>(qh, out);
}

}  // extern "C"
