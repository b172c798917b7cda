/*
 * websplat.h -- C ABI of the MI355X (gfx950) 3D Gaussian Splatting render path.
 *
 * The library implements the per-frame path that WebSplatter (arXiv
 * 2602.03207) accelerates, as a tile-based compute pipeline:
 *
 *   ws_preprocess       projection of each 3D Gaussian to a 2D splat (EWA,
 *                       Sec. 2.1 Eq. 1-2), view-dependent SH colour (Eq. 3),
 *                       opacity and bounding-box culling (Sec. 3.2, Sec. 3.4
 *                       Eq. 7-8), then compaction into (tile | depth) keys.
 *   ws_sort, ws_sort32  stable LSD radix sort of 64-bit (or 32-bit) keys with
 *                       their 32-bit values; each pass places an element at
 *                       base_d + prefix_wg + rank_local (Sec. 3.3.2, Eq. 5-6).
 *   ws_render           per-tile front-to-back alpha compositing (Eq. 2, Eq. 4).
 *   ws_render_backward  reverse mode of ws_render and ws_preprocess.
 *
 * Conventions shared by every call
 *   - Memory: every array argument is DEVICE memory owned by the caller unless
 *     the argument says "host".  The library never allocates, frees or keeps a
 *     pointer after a call returns.  Scratch memory comes from the caller
 *     through (ws, ws_bytes); its size is given by the matching
 *     ws_*_workspace_size() call.  ws must be 256-byte aligned.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream).  Calls enqueue work and return without synchronising; they do
 *     not call hipMemset or hipMalloc, so they may be captured in a HIP graph.
 *   - Errors: argument errors are detected on the host before any work is
 *     enqueued and returned as a ws_status; ws_last_error() then holds a
 *     message (thread-local).  Conditions only the device can see (too many
 *     pairs for the caller's capacity, an expired bounded wait) are written to
 *     the caller's int32 device status word `d_status`; every later kernel
 *     that receives the same d_status exits early without writing output.
 *   - Layout: Gaussian parameters are fp32 structure-of-arrays, component
 *     major: means[3][n], log_scales[3][n], quats[4][n] (w, x, y, z; need not
 *     be normalised), opacity_logits[n], sh[3*K][n] with row k*3 + c holding
 *     SH coefficient k of colour channel c, K = (sh_degree + 1)^2.
 *     Images are fp32 planar [3][H][W] per view, views packed back to back in
 *     view order.
 *   - Multi-view: every call takes n_views cameras.  Tiles of all views share
 *     one global id space: view v owns ids [tile_offset(v),
 *     tile_offset(v) + tiles_x(v) * tiles_y(v)), tile_offset being the sum of
 *     the tile counts of the views before it; tiles are row-major in a view.
 *   - Determinism: preprocess, sort and render produce identical bits on
 *     every run and for every launch configuration (tile size, radix width,
 *     ordered or plain render).  The backward pass accumulates with
 *     floating-point atomics and is reproducible only to rounding.
 */
#ifndef WEBSPLAT_H
#define WEBSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ws_status {
    WS_OK = 0,
    WS_ERR_INVALID_ARGUMENT = 1,   /* null pointer, negative size, bad option value */
    WS_ERR_UNSUPPORTED = 2,        /* valid but not implemented (e.g. sh_degree > 3, tile size) */
    WS_ERR_WORKSPACE_TOO_SMALL = 3,
    WS_ERR_HIP = 4,                /* a HIP runtime call failed; message in ws_last_error() */
    WS_ERR_CAPACITY = 5,           /* device status only: more pairs than the key buffers hold */
    WS_ERR_SPIN_LIMIT = 6          /* device status only: a bounded inter-workgroup wait expired */
} ws_status;

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  A world point X
 * maps to camera space p = R X + t and to pixel (fx p.x/p.z + cx,
 * fy p.y/p.z + cy); the centre of pixel (i, j) is (i + 0.5, j + 0.5).
 * C is the world-space camera centre used for the SH view direction
 * d = (X - C) / |X - C| (Sec. 2.1, Eq. 3).  width, height in [1, 32767]. */
typedef struct ws_camera {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];   /* row-major world -> camera rotation */
    float t[3];
    float C[3];
    int32_t reserved;  /* must be 0 */
} ws_camera;          /* 88 bytes */

/* flags */
#define WS_FLAG_FIXED_3SIGMA     1u  /* "-RADIUS" ablation (Sec. 4.4): 3-sigma extent for every splat */
#define WS_FLAG_NO_VIEWPORT_CULL 2u  /* "-CULL" ablation (Sec. 4.4): keep splats whose AABB misses the view */
#define WS_FLAG_ORDERED_RENDER   4u  /* render: persistent workgroups take tiles from a queue, longest first
                                          (grouped by the power of two of the pair count); same images */
#define WS_FLAG_DEPTH_FIRST      8u  /* preprocess: emit pairs in (depth, view * n + id) order instead of
                                        (view * n + id) order; a stable sort of the tile bits alone
                                        [32, end_bit) then yields the full (tile, depth) order */
#define WS_FLAG_KEYS32          16u  /* with WS_FLAG_DEPTH_FIRST only: keys are uint32_t tile (or bin) ids,
                                        the high words of the 64-bit keys, without the depth word (the
                                        emission order already is the depth order); ws_sort32 on bits
                                        [0, end_bit - 32) then gives the same lists; ws_render and
                                        ws_expand_bins read such keys */
#define WS_FLAG_PACKED          64u  /* packed render inputs (Sec. 3.2): ws_preprocess writes ws_splat_packed
                                        records (32 bytes: fp16 ellipse axes, RGBA8 colour and opacity)
                                        where `splats` is passed, and ws_expand_bins / ws_render read them;
                                        colours are clamped to [0, 1] and opacity, colour and the ellipse are
                                        quantised.  Forward only: ws_render_backward rejects the flag. */
#define WS_FLAG_ACCUMULATE_GRADS 32u  /* ws_render_backward: add the gradients to `grads` instead of
                                         overwriting them (a batch rendered by several calls, e.g. one view
                                         each, then sums its gradients in the library) */

typedef struct ws_options {
    int32_t tile_w, tile_h;   /* 16x16 (default), 8x8, 16x8 or 32x16 pixels */
    int32_t sh_degree;        /* 0..3 */
    int32_t radix_bits;       /* ws_sort digit width 1..10; 0 = library default (8) */
    uint32_t flags;           /* WS_FLAG_* */
    float near_z;             /* cull p.z <= near_z (default 0.2) */
    float lowpass;            /* added to both diagonal entries of the 2D covariance (0.3 px^2) */
    float clamp_fov;          /* Jacobian uses x/z, y/z clamped to clamp_fov * half-FOV tangent (1.3) */
    float alpha_min;          /* cull sigma < alpha_min; skip splats with alpha < alpha_min (1/255) */
    float alpha_max;          /* alpha = min(alpha_max, sigma exp(power)) (0.99) */
    float t_min;              /* stop before the transmittance falls below t_min (1e-4) */
    float bg[3];              /* background colour, weighted by the final transmittance */
    int32_t bin_x, bin_y;     /* key cells ("bins") of bin_x x bin_y tiles, each 1, 2, 4 or 8 (0 reads as 1).
                                 With 1 x 1 the pair keys name tiles.  With larger bins ws_preprocess keys
                                 name bins (ids laid out like tile ids, over bins of bin_x * tile_w by
                                 bin_y * tile_h pixels), tiles_touched counts bins, ws_sort orders the bin
                                 bits, and ws_expand_bins turns each bin's list into the lists of its tiles
                                 for ws_render and ws_render_backward.  Images do not change.
                                 Coverage mask: let b = ceil(log2(ws_total_bins)), at least 1.  If
                                 b + bin_x * bin_y <= 32, the key's cell word (the high word of a 64-bit
                                 key, a 32-bit key itself) holds the bin id in bits [0, b) and, above it,
                                 bit b + row * bin_x + col set for each tile (col, row) of the bin that the
                                 splat's rectangle meets; the sort must then order bits [0, b) of the cell
                                 word only (ws_sort on [32, 32 + b), ws_sort32 on [0, b)). */
} ws_options;

typedef struct ws_gaussians {
    int64_t n;                    /* number of Gaussians, 0 <= n < 2^31 */
    const float* means;           /* [3][n] */
    const float* log_scales;      /* [3][n] */
    const float* quats;           /* [4][n] */
    const float* opacity_logits;  /* [n] */
    const float* sh;              /* [3*K][n] */
} ws_gaussians;

/* One projected splat (one per view and Gaussian), 48 bytes, 16-byte aligned.
 * Valid only where tiles_touched != 0; otherwise the contents are unspecified. */
typedef struct ws_splat {
    float mean2d[2];     /* projected centre, pixels */
    float conic[3];      /* A, B, C: inverse 2D covariance [[A, B], [B, C]] */
    float opacity;       /* sigma = sigmoid(logit) */
    float rgb[3];        /* max(0, SH + 0.5) */
    float depth;         /* camera-space z, rounded to fp32 (its bits are the low key word) */
    uint16_t rect[4];    /* inclusive pixel rectangle x0, x1, y0, y1 (the culling AABB, clipped) */
} ws_splat;

/* The packed record of WS_FLAG_PACKED, 32 bytes, 16-byte aligned (Sec. 3.2
 * packs the ellipse axes as fp16 pairs and colour plus opacity as RGBA8).
 * Let Sigma' = [[a, b], [b, c]] be the projected covariance with eigenvalues
 * l1 >= l2 and unit eigenvector v1 = (x, y) of l1 (from (l1 - c, b) when
 * a >= c, else (b, l1 - a); (1, 0) when Sigma' is a multiple of I) and
 * v2 = (-y, x).  The axes are sqrt(l1) v1 and sqrt(l2) v2, each component
 * rounded to IEEE fp16 (nearest even).  The renderer uses the quantised
 * ellipse Sigma'_q = axis1 axis1^T + axis2 axis2^T, whose determinant is
 * (axis1 x axis2)^2, and its inverse as the conic.  r, g, b =
 * floor(255 min(1, colour) + 1/2), a = floor(255 sigma + 1/2); colour and
 * sigma are these bytes / 255.  Valid only where tiles_touched != 0. */
typedef struct ws_splat_packed {
    float mean2d[2];     /* projected centre, pixels */
    uint16_t axes[4];    /* fp16 bits: axis1.x, axis1.y, axis2.x, axis2.y (pixels) */
    uint8_t rgba[4];
    float depth;         /* camera-space z (fp32), as in ws_splat */
    uint16_t rect[4];    /* inclusive pixel rectangle x0, x1, y0, y1, as in ws_splat */
} ws_splat_packed;

typedef struct ws_gaussian_grads {  /* same shapes as ws_gaussians; overwritten, not accumulated */
    float* means;
    float* log_scales;
    float* quats;
    float* opacity_logits;
    float* sh;
} ws_gaussian_grads;

/* ------------------------------------------------------------------ sizes */

/* Bytes of workspace for ws_preprocess with n Gaussians, n_views views, key
 * buffers of `capacity` pairs and the given option flags. */
size_t ws_preprocess_workspace_size(int64_t n, int32_t n_views, int64_t capacity, uint32_t flags);

/* Bytes of workspace for ws_sort of up to `capacity` pairs on bits
 * [begin_bit, end_bit) with digits of radix_bits (0 = default). */
size_t ws_sort_workspace_size(int64_t capacity, int32_t begin_bit, int32_t end_bit, int32_t radix_bits);

/* The same for ws_sort32 (end_bit <= 32). */
size_t ws_sort32_workspace_size(int64_t capacity, int32_t begin_bit, int32_t end_bit, int32_t radix_bits);

/* Bytes of workspace for ws_render over these host cameras. */
size_t ws_render_workspace_size(const ws_camera* cams, int32_t n_views, const ws_options* opt);

/* Bytes of workspace for ws_render_backward. */
size_t ws_render_backward_workspace_size(int64_t n, int32_t n_views);

/* Total tile count of the views (the length of the tile_ranges array / 2). */
int64_t ws_total_tiles(const ws_camera* cams, int32_t n_views, const ws_options* opt);

/* Total key-cell count of the views: bins of bin_x x bin_y tiles (equal to
 * ws_total_tiles with 1 x 1 bins).  The pair keys' high words lie below it. */
int64_t ws_total_bins(const ws_camera* cams, int32_t n_views, const ws_options* opt);

/* Bytes of workspace for ws_expand_bins over these host cameras. */
size_t ws_expand_bins_workspace_size(const ws_camera* cams, int32_t n_views, const ws_options* opt);

/* Total image floats of the views: sum of 3 * width * height. */
int64_t ws_total_image_floats(const ws_camera* cams, int32_t n_views);

/* ------------------------------------------------------------ the path */

/* Pre-processing and key emission (Sec. 3.2; culling rules of Sec. 3.4).
 *   g           Gaussians (device arrays, see the layout above)
 *   cams        host array of n_views cameras (read during the call, for sizes)
 *   d_cams      device copy of the same n_views cameras (read by the kernels)
 *   splats      out [n_views][n] ws_splat (ws_splat_packed with WS_FLAG_PACKED)
 *   tiles_touched out [n_views][n] uint32: tiles (bins, with bins larger than
 *               one tile) covered by the splat, 0 if culled
 *   keys, values out [capacity]: pair j = ((global tile or bin id) << 32 | fp32
 *               bits of depth, Gaussian id), emitted for views in order, Gaussians
 *               in id order and tiles row-major inside each splat's rectangle.
 *               keys is uint64_t[capacity], or uint32_t[capacity] holding the
 *               tile (bin) id alone with WS_FLAG_KEYS32
 *   d_num_pairs out device int64: the number of pairs M (also when M > capacity)
 *   d_status    in/out device int32: the frame's status word.  The call's first
 *               kernel sets it to 0 (a frame starts clean); it is set to
 *               WS_ERR_CAPACITY when M > capacity (pairs beyond capacity are not
 *               written), and the later calls of the frame report into it.
 * Culls (no pair): sigma < alpha_min, p.z <= near_z, non-finite parameters or
 * zero quaternion, and a pixel rectangle that contains no pixel centre. */
ws_status ws_preprocess(const ws_gaussians* g, const ws_camera* cams, const ws_camera* d_cams, int32_t n_views,
                        const ws_options* opt, ws_splat* splats, uint32_t* tiles_touched, void* keys,
                        uint32_t* values, int64_t capacity, int64_t* d_num_pairs, int32_t* d_status, void* ws,
                        size_t ws_bytes, void* stream);

/* Stable LSD radix sort of (key, value) pairs on key bits [begin_bit, end_bit)
 * (Sec. 3.3.2): the result equals a stable sort by (key >> begin_bit) masked to
 * end_bit - begin_bit bits; values move with their keys.
 *   keys_in, values_in   input, not modified
 *   keys_out, values_out output; must not overlap the inputs
 *   n          number of pairs, or the capacity when d_n != NULL
 *   d_n        optional device int64 count (clamped to n), for device-sized sorts
 *   d_status   optional device status word: if non-zero on entry nothing is done
 * 0 <= begin_bit < end_bit <= 64; n < 2^30; 0 <= radix_bits <= 10 (0: 8).
 * With radix_bits r the sort runs ceil((end_bit - begin_bit) / r) passes; for
 * inputs of up to 2^20 pairs (the look-back schedule) r is first narrowed
 * until the histograms of all passes hold at most 2048 bins (the result is the
 * same stable order at any r). */
ws_status ws_sort(const uint64_t* keys_in, const uint32_t* values_in, uint64_t* keys_out, uint32_t* values_out,
                  int64_t n, const int64_t* d_n, const int32_t* d_status, int32_t begin_bit, int32_t end_bit,
                  int32_t radix_bits, void* ws, size_t ws_bytes, void* stream);

/* ws_sort without a workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same contract and kernels as ws_sort, for n <= 2^20 pairs (n
 * is the capacity when d_n != NULL); larger n returns WS_ERR_INVALID_ARGUMENT
 * with a message.  Its scratch memory is a 24 MiB device array inside the
 * library, one per GPU, held until the process ends; the call allocates
 * nothing (no hipMalloc, no hipFree).  Every call on a GPU uses that GPU's one
 * array, so calls that overlap in time on one GPU (different streams or
 * threads) race: serialise them.  The first call on a device looks the
 * array's address up (once per device). */
ws_status ws_sort_noalloc(const uint64_t* keys_in, const uint32_t* values_in, uint64_t* keys_out,
                          uint32_t* values_out, int64_t n, const int64_t* d_n, const int32_t* d_status,
                          int32_t begin_bit, int32_t end_bit, int32_t radix_bits, void* stream);

/* ws_sort on 32-bit keys (Sec. 3.3.2), e.g. the tile ids of WS_FLAG_KEYS32 or
 * fp32 depth bits: same contract, 0 <= begin_bit < end_bit <= 32. */
ws_status ws_sort32(const uint32_t* keys_in, const uint32_t* values_in, uint32_t* keys_out, uint32_t* values_out,
                    int64_t n, const int64_t* d_n, const int32_t* d_status, int32_t begin_bit, int32_t end_bit,
                    int32_t radix_bits, void* ws, size_t ws_bytes, void* stream);

/* Per-tile lists from bin-sorted pairs, for options with bins larger than
 * one tile (Sec. 3.2: a tile's list holds the splats whose footprint meets the
 * tile, in depth order).  A bin's pairs are contiguous after the sort and in
 * key order; every tile of the bin keeps, in that order, the pairs whose pixel
 * rectangle meets the tile.  The result is the same ids in the same order as
 * the tile's run of pairs when the keys name tiles.
 *   splats        [n_views][n] from ws_preprocess (their pixel rectangles decide;
 *                 ws_splat_packed records with WS_FLAG_PACKED)
 *   keys, values  pairs from ws_sort over the bin bits (ws_sort32 with
 *                 WS_FLAG_KEYS32); count = min(*d_num_pairs, capacity)
 *   tile_values   out [tile_capacity] uint32: every tile's list of Gaussian ids.
 *                 Each bin reserves its pair count once per tile of the bin,
 *                 so tile_capacity >= bin_x * bin_y * capacity is required
 *                 (and tile_capacity < 2^32); slots past a tile's end are
 *                 left unwritten.
 *   tile_ranges   out [total_tiles][2] uint32: [start, end) of each tile's list
 * tile_values / tile_ranges then go to ws_render (keys = NULL) and to
 * ws_render_backward as its values / tile_ranges. */
ws_status ws_expand_bins(const ws_splat* splats, int64_t n, const ws_camera* cams, const ws_camera* d_cams,
                         int32_t n_views, const ws_options* opt, const void* keys, const uint32_t* values,
                         int64_t capacity, const int64_t* d_num_pairs, const int32_t* d_status,
                         uint32_t* tile_values, int64_t tile_capacity, uint32_t* tile_ranges, void* ws,
                         size_t ws_bytes, void* stream);

/* Tile ranges and front-to-back compositing (Eq. 2, Eq. 4).
 *   splats        [n_views][n] from ws_preprocess (ws_splat_packed records with
 *                 WS_FLAG_PACKED: the ellipse, colour and opacity they quantise)
 *   keys, values  tile-sorted pairs from ws_sort (uint64_t keys) or ws_sort32
 *                 (uint32_t keys, WS_FLAG_KEYS32); count = min(*d_num_pairs, capacity).
 *                 keys = NULL: tile_ranges is an input instead (from
 *                 ws_expand_bins, with values = its tile_values and capacity
 *                 = its tile_capacity); required with bins larger than one tile
 *   tile_ranges   out [total_tiles][2] uint32: [start, end) of each tile's pairs
 *   images        out: views packed back to back, each [3][H][W] fp32
 * Per pixel, splats are taken in key order: a splat is skipped if the pixel is
 * outside its rectangle or alpha < alpha_min; the pixel stops before a splat
 * that would bring the transmittance below t_min; output = C + T * bg. */
ws_status ws_render(const ws_splat* splats, int64_t n, const ws_camera* cams, const ws_camera* d_cams,
                    int32_t n_views, const ws_options* opt, const void* keys, const uint32_t* values,
                    int64_t capacity, const int64_t* d_num_pairs, const int32_t* d_status, uint32_t* tile_ranges,
                    float* images, void* ws, size_t ws_bytes, void* stream);

/* Reverse mode of ws_render and ws_preprocess.  Given dL/dimages (same
 * layout as images), writes dL/d(parameters) summed over the views into
 * `grads` (overwritten).  The compositing adjoint recomputes each tile front
 * to back with the forward's arithmetic and decisions, and takes the colour
 * behind each splat from the forward's output `images` (its final colour
 * minus what the splats up to that one composited); the forward stores no
 * per-pixel state.  Discrete decisions (culls, skips, early stop, clamps) take
 * the derivative of the branch taken.  values / tile_ranges are the lists
 * ws_render read (with bins larger than one tile: ws_expand_bins' tile_values
 * / tile_ranges); images is ws_render's output for them.  With
 * WS_FLAG_ACCUMULATE_GRADS in opt->flags the gradients are added to `grads`
 * instead.  d_status: the forward's status word; if it is non-zero (the
 * forward did not complete) no kernel writes anything, `grads` included.
 *   tiles_touched  ws_preprocess's [n_views][n] counts for these splats, or
 *                  NULL.  The adjoint keeps one 64-byte gradient record per
 *                  (view, Gaussian) in ws; with the counts it clears and reads
 *                  only the records of entries with a non-zero count (the
 *                  only ones a tile list can hold), with NULL every record. */
ws_status ws_render_backward(const ws_gaussians* g, const ws_camera* cams, const ws_camera* d_cams,
                             int32_t n_views, const ws_options* opt, const ws_splat* splats,
                             const uint32_t* tiles_touched, const uint32_t* values, const uint32_t* tile_ranges, const float* images,
                             const float* dL_dimages, const int32_t* d_status, ws_gaussian_grads* grads, void* ws,
                             size_t ws_bytes, void* stream);

/* The compositing adjoint of the L1 photometric loss, for the training step:
 * the result of ws_l1_loss over these views' images followed by
 * ws_render_backward with its dL/dimages, without that gradient image.  The
 * adjoint forms each pixel's dL/dC = sign(images - targets) / total (sign(0) =
 * 0, 1 / total rounded once from fp64, as ws_l1_loss) from the two images,
 * and every tile sums |images - targets| over its pixels.
 *   images    the forward's images of these views (ws_render's output)
 *   targets   same layout
 *   total     element count the mean is taken over: 0 means the views'
 *             3 * sum(W * H); a larger count for a batch split over calls
 *   d_loss    out, device float: sum |images - targets| / total (per-tile fp64
 *             sums reduced in a fixed order, rounded once: identical bits run
 *             to run; it may differ from ws_l1_loss's value in the last bit,
 *             which sums in another order)
 * Every other argument, the gradients written and the status handling are
 * those of ws_render_backward; with d_status non-zero *d_loss is not written.
 * ws: ws_render_backward_l1_workspace_size bytes. */
ws_status ws_render_backward_l1(const ws_gaussians* g, const ws_camera* cams, const ws_camera* d_cams,
                                int32_t n_views, const ws_options* opt, const ws_splat* splats,
                                const uint32_t* tiles_touched, const uint32_t* values, const uint32_t* tile_ranges, const float* images,
                                const float* targets, int64_t total, float* d_loss, const int32_t* d_status,
                                ws_gaussian_grads* grads, void* ws, size_t ws_bytes, void* stream);
size_t ws_render_backward_l1_workspace_size(int64_t n, const ws_camera* cams, int32_t n_views,
                                           const ws_options* opt);

/* L1 photometric loss of the multi-view training step (the mean over every
 * image element of the batch).  Over the n floats of this call:
 *   *d_loss    = sum |images - targets| / total
 *   dL_dimages = sign(images - targets) / total        (sign(0) = 0)
 * total is the element count of the whole batch the mean is taken over
 * (total >= n); 0 means n.  A batch split over several calls (say one view
 * each) passes the batch's count to every call: the *d_loss values then add
 * up to the batch loss and the gradients are those of the batch loss.
 * Deterministic (fixed-order reduction in fp64, rounded once to fp32). */
ws_status ws_l1_loss(const float* images, const float* targets, int64_t n, int64_t total, float* dL_dimages,
                     float* d_loss, void* ws, size_t ws_bytes, void* stream);
size_t ws_l1_loss_workspace_size(int64_t n);

/* ----------------------------------------------------------- HIP graphs */

typedef struct ws_graph_s* ws_graph;

/* Begin capturing the work enqueued on `stream` (thread-local capture mode). */
ws_status ws_graph_begin(void* stream);
/* End the capture and instantiate it; *out receives an executable graph. */
ws_status ws_graph_end(void* stream, ws_graph* out);
ws_status ws_graph_launch(ws_graph graph, void* stream);
ws_status ws_graph_destroy(ws_graph graph);

/* ------------------------------------------------------- kernel timing */

/* Kernels that ws_timing_start can time. */
#define WS_KERNEL_PREPROCESS     0  /* projection, colour, culling */
#define WS_KERNEL_SCAN_EMIT      1  /* prefix sum of tile counts and key emission */
#define WS_KERNEL_SORT_HIST      2  /* digit histograms of all passes */
#define WS_KERNEL_SORT_PASS      3  /* one digit pass of the radix sort */
#define WS_KERNEL_RANGES         4  /* per-tile ranges (clear + boundaries) */
#define WS_KERNEL_RENDER         5  /* tile compositing */
#define WS_KERNEL_RENDER_BWD     6  /* compositing adjoint */
#define WS_KERNEL_PREPROCESS_BWD 7  /* preprocess adjoint */

/* While started, every launch of kernel `kernel` made by this process is
 * bracketed by two HIP events recorded on the launch's stream (up to 4096
 * launches).  ws_timing_stop waits for those events and returns the summed
 * elapsed milliseconds and the number of launches, then stops timing.  Meant
 * for benchmarks: not thread-safe, not for use under graph capture. */
ws_status ws_timing_start(int32_t kernel);
ws_status ws_timing_stop(double* total_ms, int64_t* launches);

/* ------------------------------------------------------------ utilities */

const char* ws_last_error(void);           /* thread-local message of the last failed call */
const char* ws_status_string(int32_t status);
int32_t ws_version(void);                  /* major * 10000 + minor * 100 + patch */

#ifdef __cplusplus
}
#endif

#endif /* WEBSPLAT_H */
