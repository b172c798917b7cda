// Reverse mode of the render path.
//
// k_render_bwd<TW, TH>  per tile, no stored per-pixel state: one pass walks the
//     tile's list front to back exactly as the forward does (same staged
//     arithmetic, same decisions, so T_k is the forward's transmittance) and
//     forms for each splat a pixel takes
//        dL/dc_k     = w_k dL/dC              (w_k = T_k - T_{k+1}, the forward's weight)
//        dL/dalpha_k = dL/dC . (c_k T_k - R_k / (1 - alpha_k))
//     with R_k = sum_{i>k} c_i w_i + bg T_final, the colour behind splat k,
//     taken as C - sum_{i<=k} c_i w_i from the pixel's forward output C
//     (background included): dL/dC . R_k = dL/dC . C - P_k with P_k the running
//     sum of (dL/dC . c_i) w_i
//     and, unless alpha was clamped, dL/dsigma = dL/dalpha exp(power) and
//     dL/dpower = dL/dalpha * alpha with the derivatives of the power in the
//     centre and the conic.  Per (pixel, splat) the pass forms nine values:
//     the moments dL/dpower * (1, dx, dy, dx^2, dx dy, dy^2) and the colour
//     gradient; their per-splat sums over a staged batch are reduced across
//     the wave (lane swaps and DPP), stored per wave in LDS, added over the
//     waves in a fixed order, turned into dL/d(centre, conic, sigma) with the
//     splat's conic once, and added to device memory with one atomic per
//     value.
//     With the L1 loss (L1Args.images set), dL/dC is formed in the kernel as
//     sign(image - target) / total instead of read from a gradient image, and
//     each tile writes the sum of |image - target| over its pixels (fp64, fixed
//     order) for k_l1_final.
// k_bwd_clear           zeroes the per-(view, splat) gradient buffer.
// k_preprocess_bwd_geo  one thread per Gaussian, summing over the views: the
//     chain through the conic inverse, the EWA covariance, the Jacobian
//     (branch taken at the clamp), the rotation and scale, the mean projection
//     and the sigmoid.
// k_preprocess_bwd_sh   one thread per Gaussian, summing over the views: the SH
//     colour (clamped channels give zero) and the view direction, added to the
//     mean gradient.
#include "composite.h"
#include "project.h"
#include "ws_internal.h"

namespace ws {
namespace {

constexpr int kNG = 9;  // u, v, A, B, C, sigma, r, g, b
// One 64-byte record of gradients per (view, splat): the nine values, then
// seven unused floats.  A wave adds a splat's nine values with one atomic
// instruction whose lanes address one cache line, which the memory system
// serves as one request; nine arrays would take nine.
constexpr int kRec = 16;
// (wave, entry) pairs of per-wave sums a batch holds: 64 entries per batch of
// a 16x16 tile (128 needed 18 KB of LDS per workgroup, six per CU, and 32
// doubled the batches; both were slower)
constexpr int kBwdSums = 256;

struct BwdWs {
    float* sg;   // [V * n][kRec] per-(view, splat) gradients
    int64_t vn;  // V * n
};

BwdWs carve_bwd(void* ws, int64_t n, int32_t n_views) {
    BwdWs b;
    b.vn = n * n_views;
    b.sg = static_cast<float*>(ws);
    return b;
}

// Zeroes the gradient records (recs of them, kRec / 4 float4s each), only
// those of entries with a non-zero tile count when `touched` is given: one
// thread per record reads its count once and writes the whole record.
__global__ void k_bwd_clear(float4* p, int64_t recs, const uint32_t* touched) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= recs || (touched && touched[r] == 0u)) return;
#pragma unroll
    for (int k = 0; k < kRec / 4; ++k) p[r * (kRec / 4) + k] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// The L1 loss inside the compositing adjoint (targets == nullptr: dL is read).
struct L1Args {
    const float* targets;
    float inv_total;  // 1 / total rounded once from fp64, as ws_l1_loss
    double* partial;  // [total_tiles] sums of |image - target| per tile
};

struct BwdArgs {
    const ws_splat* splats;
    int64_t n;
    const ws_camera* cams;
    int32_t n_views;
    const uint32_t* values;
    const uint32_t* ranges;
    const float* images;  // the forward's images
    const float* dL;
    L1Args l1;
    const int32_t* d_status;
    BwdWs w;
    KOpts o;
};

struct RawConic {
    float A, B, C, inv_sigma;
};

// Sums over the 64 lanes of a wave of the nine per-splat gradient values,
// transposed so that the work halves at every step: the 32-lane swap pairs up
// values (v0, v1), (v2, v3), ... and one add leaves each value's half-sums in
// one half of the wave; the 16-lane swap pairs up those and one add leaves each
// value's quarter-sums in one row (rows 0-3 hold v0, v2, v1, v3 in one
// register and v4, v6, v5, v7 in the other); two DPP adds limited to lane banks
// fold the two registers into one, the first value in lanes 0-7 of each row
// and the second in lanes 8-15; three DPP adds inside each half-row finish the
// sums.  The ninth value has no partner: the same three DPP adds and an 8-lane
// rotation sum it over each row, and two row broadcasts add the rows.
// Result: lane 8h + 16r (h = 0, 1; r = 0..3) holds the sum of value
// 4h + (0, 2, 1, 3)[r] in *q, and every lane of row 3 the sum of v8 in *q8.
// Every step is a VALU operation on all 64 lanes (the callers run with all
// lanes active); no LDS traffic.
__device__ __forceinline__ void swap32(float& a, float& b) {
    // both operands are read and written (the swap builtin of this compiler
    // returns the first register twice); two wait states on either side
    asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1\n\ts_nop 1" : "+v"(a), "+v"(b));
}
__device__ __forceinline__ void swap16(float& a, float& b) {
    asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1\n\ts_nop 1" : "+v"(a), "+v"(b));
}
template <int CTRL>
__device__ __forceinline__ float dpp_add(float v) {
    const int moved = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false);
    return v + __builtin_bit_cast(float, moved);
}
// Lanes 0-7 of each row: x + x rotated by 8 lanes (the sum of x over lanes i
// and i + 8); lanes 8-15: the same of y.  Each add writes only its two lane
// banks; a DPP source needs two wait states after the VALU write of it, and
// the result as well before the next DPP reads it.
__device__ __forceinline__ float fold_halves(float x, float y) {
    float z;
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %1, %1 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %0, %2, %2 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
        "s_nop 1"
        : "=&v"(z)
        : "v"(x), "v"(y));
    return z;
}
// The sum over each 8-lane half of a row, in all its lanes.
__device__ __forceinline__ float half_row_sum(float v) {
    v = dpp_add<0x141>(v);  // row_half_mirror: lanes i and 7 - i
    v = dpp_add<0x4e>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_add<0xb1>(v);   // quad_perm [1, 0, 3, 2]
    return v;
}
__device__ __forceinline__ void wave_sum9(float (&v)[kNG], float* q, float* q8) {
    swap32(v[0], v[1]);
    swap32(v[2], v[3]);
    swap32(v[4], v[5]);
    swap32(v[6], v[7]);
    float p01 = v[0] + v[1], p23 = v[2] + v[3], p45 = v[4] + v[5], p67 = v[6] + v[7];
    swap16(p01, p23);
    swap16(p45, p67);
    // v8 opaque: otherwise the compiler folds its product into the first DPP
    // add as a zeroed register, a DPP move and a multiply-add
    asm volatile("" : "+v"(v[8]));
    // v8: the sum over each row (half-rows and one 8-lane rotation), then
    // row_bcast:15 adds the last lane of each row to the next row (row 0 has
    // no source and adds 0) and row_bcast:31 adds lane 31 to rows 2 and 3:
    // row 3 then holds r3 + r2 + (r1 + r0)
    float s = half_row_sum(fold_halves(p01 + p23, p45 + p67));
    float s8 = dpp_add<0x143>(dpp_add<0x142>(dpp_add<0x128>(half_row_sum(v[8]))));
    // complete the sums in every lane here: left to itself the compiler moves
    // the last add of each into the storing lanes' branch, which turns one DPP
    // add into a zeroed register, a DPP move and an add
    asm volatile("" : "+v"(s), "+v"(s8));
    *q = s;
    *q8 = s8;
}

// RECT: the rectangle test of the forward (see blend_one).
template <int TW, int TH, bool RECT>
__global__ __launch_bounds__(TW * TH, 8) void k_render_bwd(BwdArgs a) {
    constexpr int NT = TW * TH, NW = NT / kWave;
    // batches of NB list entries: at most half a tile's threads, and at most
    // kBwdSums (wave, entry) pairs of per-wave sums
    constexpr int NB = NT / 2 < kBwdSums / NW ? NT / 2 : kBwdSums / NW;
    __shared__ StagedSplat s_batch[NB];
    __shared__ RawConic s_conic[NB];
    // per wave and batch entry the wave's nine sums, [wave][entry][9]: each
    // wave writes its own (a plain store, no LDS atomics), the flush adds the
    // waves' sums in a fixed order
    __shared__ float4 s_sums4[NW * NB * kNG / 4];
    float* const s_sums = reinterpret_cast<float*>(s_sums4);
    __shared__ uint64_t s_masks[NW * NW];
    __shared__ double s_l1[NW];
    if (*a.d_status != 0) return;
    const int64_t g = blockIdx.x;
    const TileInfo ti = locate_tile(a.cams, a.n_views, g, TW, TH);
    int px, py;
    quadrant_pixel<TW>(ti.x0, ti.y0, &px, &py);
    const bool inside = px < ti.W && py < ti.H;
    const bool l1 = a.l1.targets != nullptr;
    // per pixel: the forward's colour C (background included) and dL/dC, given
    // or, with the L1 loss, sign(C - target) / total (and |C - target| for the
    // tile's loss sum).
    float img[3] = {0.f, 0.f, 0.f}, aux[3] = {0.f, 0.f, 0.f};  // aux: the target, or dL/dC
    if (inside) {
        const int64_t plane = int64_t(ti.W) * ti.H;
        const int64_t p = ti.img_off + int64_t(py) * ti.W + px;
        const float* src = l1 ? a.l1.targets : a.dL;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            img[c] = a.images[p + c * plane];
            aux[c] = src[p + c * plane];
        }
    }
    float dLdC[3];
    double part = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float d = img[c] - aux[c];
        dLdC[c] = l1 ? (d > 0.f ? a.l1.inv_total : (d < 0.f ? -a.l1.inv_total : 0.f)) : aux[c];
        part += double(fabsf(d));
    }
    // dL/dC . C: dL/dC . R_k = SC - P_k, P_k = dL/dC . (colour composited up to splat k)
    const float SC = fmaf(dLdC[0], img[0], fmaf(dLdC[1], img[1], dLdC[2] * img[2]));
    const uint64_t* my_masks = s_masks + (threadIdx.x / kWave) * NW;
    const uint32_t start = a.ranges[2 * g], end = a.ranges[2 * g + 1];
    const ws_splat* vsplats = a.splats + int64_t(ti.view) * a.n;
    const int64_t vbase = int64_t(ti.view) * a.n;
    const float pcx = float(px) + 0.5f, pcy = float(py) + 0.5f;
    const uint32_t pix = inside ? pack_xy(px, py) : kNoPixel;
    const BlendConsts bk(a.o);
    float T = 1.f, P = 0.f;
    uint64_t active = wave_ballot(inside);  // lanes whose pixel is still compositing

    // One pass front to back over the tile's list, replaying the forward's
    // decisions with its arithmetic (so T_k is the forward's transmittance),
    // and forming the adjoint of every splat a pixel takes.
    for (uint32_t b0 = start; b0 < end; b0 += NB) {
        if (__syncthreads_count(!lane_in(active)) == NT) break;
        {
            const uint32_t idx = b0 + threadIdx.x;
            StagedSplat s = empty_splat();
            bool valid = false;
            if (threadIdx.x < NB && idx < end) {
                const uint32_t id = a.values[idx];
                valid = id < uint64_t(a.n);
                if (valid) s = stage_splat(vsplats, id);
                s_batch[threadIdx.x] = s;
                const float* rec = reinterpret_cast<const float*>(vsplats + (valid ? id : 0));
                s_conic[threadIdx.x] = RawConic{rec[2], rec[3], rec[4], 1.f / rec[5]};
            }
            for (int i = threadIdx.x; i < NW * NB * kNG / 4; i += NT) s_sums4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            stage_quadrant_masks<TW, TH>(s, valid, ti.x0, ti.y0, bk.log2_amin, s_masks);
        }
        __syncthreads();
        if (active != 0) {
            // front to back over the staged splats that meet this wave's quadrant
            MaskWalk<NW, true> walk;
            walk.init(my_masks);
            // The wave's nine sums of a splat are stored by nine lanes: the
            // first lane of each half-row stores its value's sum (rows hold
            // v0, v2, v1, v3, plus 4 in the second half-row), lane 49 that of v8.
            const uint32_t lane = lane_id();
            const bool leader = (lane & 7) == 0, lane49 = lane == 49;
            const int row = int(lane >> 4);
            const int kq = lane49 ? 8 : (row == 1 ? 2 : (row == 2 ? 1 : row)) + int(lane & 8) / 2;
            float* const my_sums = s_sums + (threadIdx.x / kWave) * NB * kNG + kq;
            for (int t = walk.next(); t >= 0; t = walk.next()) {
                const StagedSplat s = s_batch[t];
                // the forward's evaluation and decisions (blend_one), as lane masks
                const float dx = s.u - pcx, dy = s.v - pcy;
                const float araw = raw_alpha(s, dx, dy);
                const float alpha = __builtin_amdgcn_fmed3f(araw, 0.f, bk.alpha_max);
                const float Tn = fmaf(-T, alpha, T);
                const uint64_t hit = (RECT ? active & wave_ballot(in_rect(s, pix)) : active) &
                                     wave_ballot(!(alpha < bk.alpha_min));
                const uint64_t stop = hit & wave_ballot(Tn < bk.t_min);
                const uint64_t take_m = hit & ~stop;
                active &= ~stop;
                if (take_m != 0) {
                    // every lane evaluates the adjoint without branches: a lane
                    // that does not take the splat gets zero weights, so its sums
                    // and state stay unchanged
                    const bool take = lane_in(take_m);
                    const bool unclamped = lane_in(take_m & wave_ballot(!(araw > bk.alpha_max)));
                    const float T1 = take ? Tn : T;
                    const float w = T - T1;  // the forward's weight of splat k
                    const float Dc = fmaf(dLdC[0], s.r, fmaf(dLdC[1], s.g, dLdC[2] * s.b));  // dL/dC . c_k
                    P = fmaf(Dc, w, P);
                    // 1 - alpha >= 1 - alpha_max > 0 (hardware reciprocal, about 1 ulp)
                    const float inv = __builtin_amdgcn_rcpf(1.f - alpha);
                    // dL/dalpha = dL/dC . (c_k T_k - R_k / (1 - alpha)); zero through the clamp
                    const float dLda = fmaf(T, Dc, -(SC - P) * inv);
                    const float gp = unclamped ? dLda * araw : 0.f;  // dL/dpower
                    // moments of dL/dpower over the splat's pixels; the conic and
                    // 1/sigma, constant per splat, are applied once to their sums
                    // (flush below)
                    float gv[kNG];
                    const float gdx = gp * dx, gdy = gp * dy;
                    gv[0] = gdx;
                    gv[1] = gdy;
                    gv[2] = gdx * dx;
                    gv[3] = gdx * dy;
                    gv[4] = gdy * dy;
                    gv[5] = gp;
                    gv[6] = dLdC[0] * w;
                    gv[7] = dLdC[1] * w;
                    gv[8] = dLdC[2] * w;
                    T = T1;
                    float q, q8;
                    wave_sum9(gv, &q, &q8);
                    if (leader || lane49) my_sums[t * kNG] = lane49 ? q8 : q;
                }
                if (active == 0) break;
            }
        }
        __syncthreads();
        // One lane per (entry, value), sixteen lanes per entry: value k of the
        // entry's gradient record, from the waves' sums added in wave order.
        // From the moments S0..S5 of dL/dpower (with dx = u - px, dy = v - py):
        //   dL/du = -(A S0 + B S1), dL/dv = -(B S0 + C S1),
        //   dL/dA = -S2 / 2, dL/dB = -S3, dL/dC = -S4 / 2, dL/dsigma = S5 / sigma
        for (int i = threadIdx.x; i < NB * kRec; i += NT) {
            const int t = i / kRec, k = i % kRec;
            if (k >= kNG || b0 + uint32_t(t) >= end) continue;
            const uint32_t id = s_batch[t].id;
            if (id >= uint64_t(a.n)) continue;
            const float* sums = s_sums + t * kNG;
            float mk = 0.f, mo = 0.f;  // S_k, and for k < 2 S_(1-k)
#pragma unroll
            for (int w = 0; w < NW; ++w) mk += sums[w * NB * kNG + k];
            if (k < 2) {
#pragma unroll
                for (int w = 0; w < NW; ++w) mo += sums[w * NB * kNG + (1 - k)];
            }
            const RawConic q = s_conic[t];
            float gg;
            if (k == 0)
                gg = -fmaf(q.A, mk, q.B * mo);
            else if (k == 1)
                gg = -fmaf(q.B, mo, q.C * mk);
            else if (k == 2 || k == 4)
                gg = -0.5f * mk;
            else if (k == 3)
                gg = -mk;
            else if (k == 5)
                gg = mk * q.inv_sigma;
            else
                gg = mk;
            if (gg != 0.f) atomicAdd(&a.w.sg[(vbase + id) * kRec + k], gg);
        }
    }
    if (l1) {
        // the tile's sum of |image - target| (lanes without a pixel hold zeros)
        part = wave_sum(part);
        if (lane_id() == 0) s_l1[threadIdx.x / kWave] = part;
        __syncthreads();
        if (threadIdx.x == 0) {
            double sum = 0.0;
            for (int w = 0; w < NW; ++w) sum += s_l1[w];
            a.l1.partial[g] = sum;
        }
    }
}

struct PreBwdArgs {
    GaussPtrs g;
    const ws_camera* cams;
    int32_t n_views;
    KOpts o;
    BwdWs w;
    const uint32_t* touched;  // [V][n] tile counts, or nullptr: every record was cleared
    GradPtrs out;
    const int32_t* d_status;
};

// A gradient value written out: stored, or added to the caller's value with
// WS_FLAG_ACCUMULATE_GRADS.
__device__ __forceinline__ void put_grad(float* p, float v, bool acc) { *p = acc ? *p + v : v; }

// Derivatives of the rotation matrix of a unit quaternion (w, x, y, z):
// returns sum_ij G_ij dR_ij/dq_c for c = w, x, y, z.
__device__ __forceinline__ void rotmat_vjp(const float* q, const float* G, float* gq) {
    const float w = q[0], x = q[1], y = q[2], z = q[3];
    // R = [[1-2(yy+zz), 2(xy-wz), 2(xz+wy)], [2(xy+wz), 1-2(xx+zz), 2(yz-wx)], [2(xz-wy), 2(yz+wx), 1-2(xx+yy)]]
    gq[0] = 2.f * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
    gq[1] = 2.f * (y * G[1] + z * G[2] + y * G[3] - 2.f * x * G[4] - w * G[5] + z * G[6] + w * G[7] -
                   2.f * x * G[8]);
    gq[2] = 2.f * (-2.f * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] -
                   2.f * y * G[8]);
    gq[3] = 2.f * (-2.f * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.f * z * G[4] + y * G[5] + x * G[6] +
                   y * G[7]);
}

// Geometry part of the pre-processing adjoint: per Gaussian, over the views in
// which its centre, conic or opacity received a gradient.
template <int DEG>
__global__ __launch_bounds__(128) void k_preprocess_bwd_geo(PreBwdArgs a) {
    const int64_t i = int64_t(blockIdx.x) * 128 + threadIdx.x;
    const int64_t n = a.g.n;
    if (i >= n || *a.d_status != 0) return;
    float gm[3] = {0.f, 0.f, 0.f}, gls[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f}, glogit = 0.f;
    for (int32_t v = 0; v < a.n_views; ++v) {
        const int64_t vi = int64_t(v) * n + i;
        if (a.touched && a.touched[vi] == 0u) continue;  // in no tile list: no gradient, record not cleared
        const float4* rec = reinterpret_cast<const float4*>(a.w.sg + vi * kRec);
        const float4 r0 = rec[0], r1 = rec[1];
        const float gs[6] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y};
        bool any = false;
#pragma unroll
        for (int k = 0; k < 6; ++k) any = any || gs[k] != 0.f;
        if (!any) continue;
        const ws_camera& cam = a.cams[v];
        ProjState st;
        if (!compute_projection<DEG, false>(a.g, i, cam, a.o, st)) continue;
        // ---- opacity
        glogit += gs[5] * st.sigma * (1.f - st.sigma);
        // ---- conic (A, B, C) = (c, -b, a) / det  ->  Sigma' entries (a, b, c)
        const float ca = st.a, cb = st.b, cc = st.c;
        const float idet = 1.f / st.det;
        const float idet2 = idet * idet;
        const float gA = gs[2], gB = gs[3], gC = gs[4];
        const float ga = (-gA * cc * cc + gB * cb * cc - gC * cb * cb) * idet2;
        const float gb = (2.f * gA * cb * cc - gB * (ca * cc + cb * cb) + 2.f * gC * ca * cb) * idet2;
        const float gc2 = (-gA * cb * cb + gB * ca * cb - gC * ca * ca) * idet2;
        // ---- Sigma' = M M^T + lowpass I
        const float* M = st.M;
        float gM[6];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            gM[j] = 2.f * ga * M[j] + gb * M[3 + j];
            gM[3 + j] = gb * M[j] + 2.f * gc2 * M[3 + j];
        }
        // ---- M = J (T S), T = W Rq
        const float iz = st.invz;
        const float j00 = cam.fx * iz, j02 = -cam.fx * st.rxc * iz;
        const float j11 = cam.fy * iz, j12 = -cam.fy * st.ryc * iz;
        float gT[9];
        float gj00 = 0.f, gj02 = 0.f, gj11 = 0.f, gj12 = 0.f;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float sj = st.s[j];
            const float m0 = j00 * st.T[j] + j02 * st.T[6 + j];
            const float m1 = j11 * st.T[3 + j] + j12 * st.T[6 + j];
            gls[j] += (gM[j] * m0 + gM[3 + j] * m1) * sj;  // d/dlog s = s d/ds
            gT[j] = gM[j] * j00 * sj;
            gT[3 + j] = gM[3 + j] * j11 * sj;
            gT[6 + j] = (gM[j] * j02 + gM[3 + j] * j12) * sj;
            gj00 += gM[j] * st.T[j] * sj;
            gj02 += gM[j] * st.T[6 + j] * sj;
            gj11 += gM[3 + j] * st.T[3 + j] * sj;
            gj12 += gM[3 + j] * st.T[6 + j] * sj;
        }
        // ---- T = W Rq  ->  dL/dRq = W^T dL/dT
        float gR[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                gR[r * 3 + c] = cam.R[0 * 3 + r] * gT[0 * 3 + c] + cam.R[1 * 3 + r] * gT[1 * 3 + c] +
                                cam.R[2 * 3 + r] * gT[2 * 3 + c];
        float gqh[4];
        rotmat_vjp(st.q, gR, gqh);
        {
            const float dq = gqh[0] * st.q[0] + gqh[1] * st.q[1] + gqh[2] * st.q[2] + gqh[3] * st.q[3];
            const float iq = 1.f / st.qnorm;
#pragma unroll
            for (int c = 0; c < 4; ++c) gq[c] += (gqh[c] - st.q[c] * dq) * iq;
        }
        // ---- Jacobian and mean projection -> camera-space centre p
        const float iz2 = iz * iz;
        const float rx = float(st.px / st.pz), ry = float(st.py / st.pz);
        float gpx = gs[0] * cam.fx * iz, gpy = gs[1] * cam.fy * iz;
        float gpz = -gs[0] * cam.fx * rx * iz - gs[1] * cam.fy * ry * iz;
        gpz += -gj00 * cam.fx * iz2 - gj11 * cam.fy * iz2;
        if (st.clamp & kClampJx) {
            gpz += gj02 * cam.fx * st.rxc * iz2;  // j02 = -fx rxc / z with rxc fixed
        } else {
            gpx += -gj02 * cam.fx * iz2;  // j02 = -fx x / z^2
            gpz += 2.f * gj02 * cam.fx * st.rxc * iz2;
        }
        if (st.clamp & kClampJy) {
            gpz += gj12 * cam.fy * st.ryc * iz2;
        } else {
            gpy += -gj12 * cam.fy * iz2;
            gpz += 2.f * gj12 * cam.fy * st.ryc * iz2;
        }
        // ---- p = W X + t
#pragma unroll
        for (int c = 0; c < 3; ++c) gm[c] += cam.R[0 * 3 + c] * gpx + cam.R[1 * 3 + c] * gpy + cam.R[2 * 3 + c] * gpz;
    }
    const bool acc = (a.o.flags & WS_FLAG_ACCUMULATE_GRADS) != 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        put_grad(&a.out.means[c * n + i], gm[c], acc);
        put_grad(&a.out.log_scales[c * n + i], gls[c], acc);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) put_grad(&a.out.quats[c * n + i], gq[c], acc);
    put_grad(&a.out.logits[i], glogit, acc);
}


// Colour part of the pre-processing adjoint: per Gaussian, over the views in
// which its colour received a gradient, the SH coefficient gradients (clamped
// channels give zero) and the gradient of the view direction, which it adds to
// the mean gradient written by k_preprocess_bwd_geo.  A nonzero colour
// gradient means the splat was rendered in that view, so its culling tests
// need not be repeated.  Split from the geometry part so that neither keeps
// the other's registers live across the view loop.
template <int DEG>
__global__ __launch_bounds__(128) void k_preprocess_bwd_sh(PreBwdArgs a) {
    const int64_t i = int64_t(blockIdx.x) * 128 + threadIdx.x;
    const int64_t n = a.g.n;
    if (i >= n || *a.d_status != 0) return;
    constexpr int K = (DEG + 1) * (DEG + 1);
    float gm[3] = {0.f, 0.f, 0.f};
    float gsh[3 * K];
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) gsh[k] = 0.f;
    const float mx = a.g.means[i], my = a.g.means[n + i], mz = a.g.means[2 * n + i];
    for (int32_t v = 0; v < a.n_views; ++v) {
        const int64_t vi = int64_t(v) * n + i;
        if (a.touched && a.touched[vi] == 0u) continue;
        const float* rec = a.w.sg + vi * kRec;
        const float2 rg = *reinterpret_cast<const float2*>(rec + 6);
        const float gcol[3] = {rg.x, rg.y, rec[8]};
        if (gcol[0] == 0.f && gcol[1] == 0.f && gcol[2] == 0.f) continue;
        const ws_camera& cam = a.cams[v];
        // the forward's view direction and colour (same arithmetic)
        float dx = mx - cam.C[0], dy = my - cam.C[1], dz = mz - cam.C[2];
        const float dir_norm = sqrtf(dx * dx + dy * dy + dz * dz);
        const float idn = 1.f / dir_norm;
        dx *= idn;
        dy *= idn;
        dz *= idn;
        float Y[16];
        sh_eval_basis(dx, dy, dz, DEG, Y);
        // the coefficients, read by walking one pointer down the rows: the
        // pointer is opaque to the compiler, so it does not hoist the 3K row
        // addresses out of the loop (3K 64-bit addresses held in registers
        // halved the kernel's resident waves)
        const float* p = a.g.sh + i;
        asm volatile("" : "+v"(p));
        float shc[3 * K];
#pragma unroll
        for (int k = 0; k < 3 * K; ++k) {
            shc[k] = *p;
            p += n;
        }
        float col[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) col[ch] = fmaf(shc[k * 3 + ch], Y[k], col[ch]);
        }
        float wsh[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) wsh[k] = 0.f;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float gc = col[ch] < 0.f ? 0.f : gcol[ch];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                gsh[k * 3 + ch] = fmaf(gc, Y[k], gsh[k * 3 + ch]);
                wsh[k] = fmaf(gc, shc[k * 3 + ch], wsh[k]);
            }
        }
        float gdx, gdy, gdz;
        sh_basis_vjp(dx, dy, dz, DEG, wsh, &gdx, &gdy, &gdz);
        const float dd = gdx * dx + gdy * dy + gdz * dz;
        gm[0] += (gdx - dx * dd) * idn;
        gm[1] += (gdy - dy * dd) * idn;
        gm[2] += (gdz - dz * dd) * idn;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) a.out.means[c * n + i] += gm[c];
    const bool acc = (a.o.flags & WS_FLAG_ACCUMULATE_GRADS) != 0;
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) put_grad(&a.out.sh[int64_t(k) * n + i], gsh[k], acc);
}

template <int TW, int TH>
void launch_bwd_t(const BwdArgs& ba, int64_t tiles, hipStream_t stream) {
    if (ba.o.flags & WS_FLAG_FIXED_3SIGMA)
        hipLaunchKernelGGL((k_render_bwd<TW, TH, true>), dim3(uint32_t(tiles)), dim3(TW * TH), 0, stream, ba);
    else
        hipLaunchKernelGGL((k_render_bwd<TW, TH, false>), dim3(uint32_t(tiles)), dim3(TW * TH), 0, stream, ba);
}

}  // namespace

size_t render_backward_workspace(int64_t n, int32_t n_views) {
    return align_up(size_t(kRec) * size_t(std::max<int64_t>(n, 1)) * n_views * sizeof(float));
}

size_t render_backward_l1_workspace(int64_t n, int32_t n_views, int64_t total_tiles) {
    return render_backward_workspace(n, n_views) + align_up(size_t(std::max<int64_t>(total_tiles, 1)) * sizeof(double));
}

hipError_t launch_render_backward(const GaussPtrs& g, const ws_camera* d_cams, int32_t n_views,
                                  int64_t total_tiles, const KOpts& o, const ws_splat* splats,
                                  const uint32_t* tiles_touched, const uint32_t* values, const uint32_t* tile_ranges,
                                  const float* images, const float* dL_dimages, const int32_t* d_status,
                                  const GradPtrs& grads, void* ws, hipStream_t stream, const L1Loss* l1) {
    BwdWs w = carve_bwd(ws, g.n, n_views);
    double* l1_part = l1 ? reinterpret_cast<double*>(static_cast<char*>(ws) + render_backward_workspace(g.n, n_views))
                         : nullptr;
    const uint32_t cgrid = uint32_t(std::max<int64_t>((w.vn + 255) / 256, 1));
    hipLaunchKernelGGL(k_bwd_clear, dim3(cgrid), dim3(256), 0, stream, reinterpret_cast<float4*>(w.sg), w.vn,
                       tiles_touched);
    // with no Gaussians only the loss remains (every tile list is empty)
    if (g.n == 0 && !l1) return hipGetLastError();
    if (total_tiles > 0) {
        BwdArgs ba;
        ba.splats = splats;
        ba.n = g.n;
        ba.cams = d_cams;
        ba.n_views = n_views;
        ba.values = values;
        ba.ranges = tile_ranges;
        ba.images = images;
        ba.dL = dL_dimages;
        ba.l1 = L1Args{nullptr, 0.f, nullptr};
        if (l1) ba.l1 = L1Args{l1->targets, float(1.0 / double(l1->total)), l1_part};
        ba.d_status = d_status;
        ba.w = w;
        ba.o = o;
        timing_begin(WS_KERNEL_RENDER_BWD, stream);
        if (o.tile_w == 16 && o.tile_h == 16) launch_bwd_t<16, 16>(ba, total_tiles, stream);
        else if (o.tile_w == 8 && o.tile_h == 8) launch_bwd_t<8, 8>(ba, total_tiles, stream);
        else if (o.tile_w == 16 && o.tile_h == 8) launch_bwd_t<16, 8>(ba, total_tiles, stream);
        else launch_bwd_t<32, 16>(ba, total_tiles, stream);
        timing_end(WS_KERNEL_RENDER_BWD, stream);
        if (l1) launch_l1_final(l1_part, total_tiles, l1->total, d_status, l1->d_loss, stream);
    }
    if (g.n == 0) return hipGetLastError();
    PreBwdArgs pa;
    pa.g = g;
    pa.cams = d_cams;
    pa.n_views = n_views;
    pa.o = o;
    pa.w = w;
    pa.touched = tiles_touched;
    pa.out = grads;
    pa.d_status = d_status;
    const dim3 grid(uint32_t((g.n + 127) / 128));
    timing_begin(WS_KERNEL_PREPROCESS_BWD, stream);
    // geometry first (writes the mean gradient), then colour (adds to it)
    switch (o.sh_degree) {
        case 0:
            hipLaunchKernelGGL(k_preprocess_bwd_geo<0>, grid, dim3(128), 0, stream, pa);
            hipLaunchKernelGGL(k_preprocess_bwd_sh<0>, grid, dim3(128), 0, stream, pa);
            break;
        case 1:
            hipLaunchKernelGGL(k_preprocess_bwd_geo<1>, grid, dim3(128), 0, stream, pa);
            hipLaunchKernelGGL(k_preprocess_bwd_sh<1>, grid, dim3(128), 0, stream, pa);
            break;
        case 2:
            hipLaunchKernelGGL(k_preprocess_bwd_geo<2>, grid, dim3(128), 0, stream, pa);
            hipLaunchKernelGGL(k_preprocess_bwd_sh<2>, grid, dim3(128), 0, stream, pa);
            break;
        default:
            hipLaunchKernelGGL(k_preprocess_bwd_geo<3>, grid, dim3(128), 0, stream, pa);
            hipLaunchKernelGGL(k_preprocess_bwd_sh<3>, grid, dim3(128), 0, stream, pa);
            break;
    }
    timing_end(WS_KERNEL_PREPROCESS_BWD, stream);
    return hipGetLastError();
}

}  // namespace ws
