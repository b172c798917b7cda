"""fp64 CPU oracle of the 3D Gaussian Splatting render path (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, the smoke entry point and the
CPU-baseline leg of the benchmark use this package; the GPU library never
does, and the two share no code.  The arithmetic lives in oracle.cpp (plain
C++17, fp64); this module only marshals numpy arrays.  The library is built
with OpenMP: its loops over independent Gaussians, tiles and pixel rows run on
set_threads() host threads (OMP_NUM_THREADS by default) and give the same bits
for any thread count; the sort is std::stable_sort on one thread.

Every input is widened from the caller's values to fp64 before the call, so a
GPU run fed the same fp32 arrays sees exactly the same numbers.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
# ORACLE_SANITIZE=1 selects a build with AddressSanitizer and UndefinedBehaviorSanitizer (host code only;
# the process must preload the ASan runtime, e.g. LD_PRELOAD=$(g++ -print-file-name=libasan.so))
_SANITIZE = os.environ.get("ORACLE_SANITIZE", "") == "1"
_LIB_PATH = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")
_lib = None

STATUS = {"visible": 0, "opacity": 1, "near": 2, "degenerate": 3, "viewport": 4}
FLAG_FIXED_3SIGMA = 1
FLAG_NO_VIEWPORT_CULL = 2


def build(verbose=False, sanitize=None):
    """Compile oracle.cpp into liboracle.so with g++ (no GPU code involved).

    sanitize=True (default: the ORACLE_SANITIZE environment variable) builds liboracle_san.so with
    -fsanitize=address,undefined instead, any undefined behaviour being fatal."""
    sanitize = _SANITIZE if sanitize is None else sanitize
    out = os.path.join(_HERE, "liboracle_san.so" if sanitize else "liboracle.so")
    if sanitize:
        cmd = ["g++", "-O1", "-g", "-std=c++17", "-Wall", "-Wextra", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-shared", "-fPIC", "-o", out, _SRC]
    else:
        cmd = ["g++", "-O2", "-std=c++17", "-Wall", "-Wextra", "-fopenmp", "-shared", "-fPIC", "-o", out, _SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB_PATH)
    P = C.POINTER
    d, i64, i32 = P(C.c_double), C.c_int64, C.c_int32
    lib.orc_preprocess.argtypes = [i64, d, d, d, d, d, P(_Camera), P(_Options), P(_Projected)]
    lib.orc_emit.argtypes = [i64, P(_Camera), P(_Options), d, d, d, d, d, i64, P(C.c_uint64), P(C.c_uint32), i64]
    lib.orc_emit.restype = i64
    lib.orc_stable_sort.argtypes = [i64, P(C.c_uint64), P(C.c_uint32), i32, i32]
    lib.orc_tile_ranges.argtypes = [i64, P(C.c_uint64), i64, P(C.c_int64)]
    lib.orc_composite.argtypes = [i64, d, d, d, d, P(C.c_int32), P(_Camera), P(_Options), i64, P(C.c_uint32),
                                  P(C.c_int64), i64, P(C.c_uint8), P(_Image)]
    lib.orc_render_brute.argtypes = [i64, d, d, d, d, d, P(_Camera), P(_Options), P(C.c_uint8), P(_Image)]
    lib.orc_forward_backward.argtypes = [i64, d, d, d, d, d, P(_Camera), P(_Options), d, d, d, d, d, d, d, d]
    lib.orc_forward_backward.restype = C.c_uint64
    lib.orc_composite_outcomes.argtypes = [i64, d, d, d, d, P(C.c_int32), P(_Camera), P(_Options), P(C.c_uint32),
                                           P(C.c_int64), i64, P(C.c_uint8), i32, i64, P(C.c_int64), P(C.c_int32),
                                           d, d]
    lib.orc_composite_outcomes.restype = i64
    lib.orc_set_threads.argtypes = [i32]
    lib.orc_max_threads.restype = i32
    lib.orc_sh_basis.argtypes = [d, i32, d]
    lib.orc_quat_to_rotmat.argtypes = [d, d]
    _lib = lib
    return lib


class _Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("R", C.c_double * 9), ("t", C.c_double * 3),
                ("C", C.c_double * 3)]


class _Options(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("sh_degree", C.c_int32), ("flags", C.c_int32),
                ("near_z", C.c_double), ("lowpass", C.c_double), ("clamp_fov", C.c_double),
                ("alpha_min", C.c_double), ("alpha_max", C.c_double), ("t_min", C.c_double),
                ("bg", C.c_double * 3)]


class _Projected(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in (
        "status", "mean2d", "conic", "cov2d", "z", "depth32", "opacity", "rgb", "pix_rect", "tile_rect",
        "tiles_touched", "clamp_bits", "bounds")]


class _Image(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in ("rgb", "T", "n_eval", "n_contrib", "alpha_margin", "t_margin", "hash")]


@dataclass
class Options:
    """Render options; the values are the readings of the paper used throughout."""
    tile_w: int = 16
    tile_h: int = 16
    sh_degree: int = 0
    flags: int = 0
    near_z: float = 0.2
    lowpass: float = 0.3
    clamp_fov: float = 1.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    bg: tuple = (0.0, 0.0, 0.0)


def _opts(o: Options) -> _Options:
    s = _Options()
    s.tile_w, s.tile_h, s.sh_degree, s.flags = o.tile_w, o.tile_h, o.sh_degree, o.flags
    s.near_z, s.lowpass, s.clamp_fov = o.near_z, o.lowpass, o.clamp_fov
    s.alpha_min, s.alpha_max, s.t_min = o.alpha_min, o.alpha_max, o.t_min
    s.bg[:] = [float(b) for b in o.bg]
    return s


def _cam(cam) -> _Camera:
    s = _Camera()
    s.width, s.height = int(cam.width), int(cam.height)
    s.fx, s.fy, s.cx, s.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    s.R[:] = [float(x) for x in np.asarray(cam.R, dtype=np.float64).reshape(9)]
    s.t[:] = [float(x) for x in np.asarray(cam.t, dtype=np.float64).reshape(3)]
    s.C[:] = [float(x) for x in np.asarray(cam.C, dtype=np.float64).reshape(3)]
    return s


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _scene64(scene):
    return (_f64(scene.means), _f64(scene.log_scales), _f64(scene.quats), _f64(scene.opacity_logits),
            _f64(scene.sh))


def _check_opts(scene, opts: Options):
    if opts.sh_degree != scene.sh_degree:
        raise ValueError("opts.sh_degree must equal scene.sh_degree")


def preprocess(scene, cam, opts: Options) -> dict:
    """Per-Gaussian projection, colour and culling for one camera (all fp64)."""
    _check_opts(scene, opts)
    lib = _load()
    n = scene.n
    out = dict(
        status=np.zeros(n, np.int8), mean2d=np.zeros((2, n)), conic=np.zeros((3, n)), cov2d=np.zeros((3, n)),
        z=np.zeros(n), depth32=np.zeros(n, np.float32), opacity=np.zeros(n), rgb=np.zeros((3, n)),
        pix_rect=np.zeros((4, n), np.int32), tile_rect=np.zeros((4, n), np.int32),
        tiles_touched=np.zeros(n, np.int64), clamp_bits=np.zeros(n, np.uint8), bounds=np.zeros((4, n)))
    P = _Projected(**{k: out[k].ctypes.data for k in out})
    m, s, q, o, sh = _scene64(scene)
    lib.orc_preprocess(n, _dp(m), _dp(s), _dp(q), _dp(o), _dp(sh), C.byref(_cam(cam)), C.byref(_opts(opts)),
                       C.byref(P))
    return out


def tiles_xy(cam, opts: Options):
    return (cam.width + opts.tile_w - 1) // opts.tile_w, (cam.height + opts.tile_h - 1) // opts.tile_h


def emit(scene, cam, opts: Options, tile_offset=0):
    """(tile | depth) keys and Gaussian-id values in emission order."""
    _check_opts(scene, opts)
    lib = _load()
    m, s, q, o, sh = _scene64(scene)
    cam_s, opt_s = _cam(cam), _opts(opts)
    count = lib.orc_emit(scene.n, C.byref(cam_s), C.byref(opt_s), _dp(m), _dp(s), _dp(q), _dp(o), _dp(sh),
                         tile_offset, None, None, 0)
    keys = np.zeros(count, np.uint64)
    vals = np.zeros(count, np.uint32)
    lib.orc_emit(scene.n, C.byref(cam_s), C.byref(opt_s), _dp(m), _dp(s), _dp(q), _dp(o), _dp(sh), tile_offset,
                 keys.ctypes.data_as(C.POINTER(C.c_uint64)), vals.ctypes.data_as(C.POINTER(C.c_uint32)), count)
    return keys, vals


def pair_count(scene, cam, opts: Options) -> int:
    """Number of (tile, splat) pairs the view emits (the sum of tiles_touched)."""
    _check_opts(scene, opts)
    lib = _load()
    m, s, q, o, sh = _scene64(scene)
    return int(lib.orc_emit(scene.n, C.byref(_cam(cam)), C.byref(_opts(opts)), _dp(m), _dp(s), _dp(q), _dp(o),
                            _dp(sh), 0, None, None, 0))


def stable_sort(keys, vals, begin_bit=0, end_bit=64):
    """std::stable_sort of the pairs on key bits [begin_bit, end_bit); returns sorted copies."""
    lib = _load()
    k = np.array(keys, dtype=np.uint64, copy=True)
    v = np.array(vals, dtype=np.uint32, copy=True)
    lib.orc_stable_sort(k.size, k.ctypes.data_as(C.POINTER(C.c_uint64)), v.ctypes.data_as(C.POINTER(C.c_uint32)),
                        begin_bit, end_bit)
    return k, v


def tile_ranges(keys, n_tiles):
    lib = _load()
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    r = np.zeros((n_tiles, 2), np.int64)
    lib.orc_tile_ranges(k.size, k.ctypes.data_as(C.POINTER(C.c_uint64)), n_tiles,
                        r.ctypes.data_as(C.POINTER(C.c_int64)))
    return r


def _image_buffers(H, W):
    return dict(rgb=np.zeros((3, H, W)), T=np.zeros((H, W)), n_eval=np.zeros((H, W), np.int64),
                n_contrib=np.zeros((H, W), np.int64), alpha_margin=np.full((H, W), np.inf),
                t_margin=np.full((H, W), np.inf), hash=np.zeros((H, W), np.uint64))


def composite_outcomes(mean2d, conic, opacity, rgb, pix_rect, cam, opts: Options, vals, ranges, tile_offset=0,
                       mask=None, max_out=64):
    """The pixels whose compositing takes a decision within fp32 reach of its threshold (alpha_min or t_min),
    with every composite that the combinations of those decisions give (each a correct result of the rule for an
    fp32 evaluation; reading A25).  Same inputs as composite().

    Returns dict(pix [k] flat pixel indices, n_out [k] (0: more than max_out combinations, not enumerated),
    rgb [k, max_out, 3] the outcomes, bound [k] the transmittance at the pixel's first such decision times the
    largest colour of its list: no choice there can move the pixel by more)."""
    lib = _load()
    n = int(np.asarray(opacity).shape[0])
    mean2d, conic, opacity, rgb = _f64(mean2d), _f64(conic), _f64(opacity), _f64(rgb)
    pr = np.ascontiguousarray(pix_rect, dtype=np.int32)
    v = np.ascontiguousarray(vals, dtype=np.uint32)
    rg = np.ascontiguousarray(ranges, dtype=np.int64)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    cam_s, opt_s = _cam(cam), _opts(opts)

    def call(cap, pix, n_out, out_rgb, bound):
        P = C.POINTER
        return lib.orc_composite_outcomes(
            n, _dp(mean2d), _dp(conic), _dp(opacity), _dp(rgb), pr.ctypes.data_as(P(C.c_int32)), C.byref(cam_s),
            C.byref(opt_s), v.ctypes.data_as(P(C.c_uint32)), rg.ctypes.data_as(P(C.c_int64)), tile_offset,
            None if mk is None else mk.ctypes.data_as(P(C.c_uint8)), max_out, cap,
            None if pix is None else pix.ctypes.data_as(P(C.c_int64)),
            None if n_out is None else n_out.ctypes.data_as(P(C.c_int32)),
            None if out_rgb is None else _dp(out_rgb), None if bound is None else _dp(bound))

    count = int(call(0, None, None, None, None))
    pix = np.zeros(max(count, 1), np.int64)
    n_out = np.zeros(max(count, 1), np.int32)
    out_rgb = np.zeros((max(count, 1), max_out, 3))
    bound = np.zeros(max(count, 1))
    call(count, pix, n_out, out_rgb, bound)
    return dict(pix=pix[:count], n_out=n_out[:count], rgb=out_rgb[:count], bound=bound[:count])


def composite(mean2d, conic, opacity, rgb, pix_rect, cam, opts: Options, vals, ranges, tile_offset=0, mask=None,
              outcomes=False):
    """Tiled front-to-back compositing of given projected splats (fp64) and a sorted pair list.

    outcomes=True also attaches composite_outcomes() of the same inputs as out["outcomes"]."""
    lib = _load()
    n = int(np.asarray(opacity).shape[0])
    mean2d, conic, opacity, rgb = _f64(mean2d), _f64(conic), _f64(opacity), _f64(rgb)
    pr = np.ascontiguousarray(pix_rect, dtype=np.int32)
    v = np.ascontiguousarray(vals, dtype=np.uint32)
    rg = np.ascontiguousarray(ranges, dtype=np.int64)
    out = _image_buffers(cam.height, cam.width)
    img = _Image(**{k: out[k].ctypes.data for k in out})
    mk = None
    if mask is not None:
        mk = np.ascontiguousarray(mask, dtype=np.uint8)
    lib.orc_composite(n, _dp(mean2d), _dp(conic), _dp(opacity), _dp(rgb), pr.ctypes.data_as(C.POINTER(C.c_int32)),
                      C.byref(_cam(cam)), C.byref(_opts(opts)), v.size, v.ctypes.data_as(C.POINTER(C.c_uint32)),
                      rg.ctypes.data_as(C.POINTER(C.c_int64)), tile_offset,
                      None if mk is None else mk.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(img))
    if outcomes:
        out["outcomes"] = composite_outcomes(mean2d, conic, opacity, rgb, pr, cam, opts, v, rg, tile_offset, mask)
    return out


def ellipse_axes(cov2d):
    """Principal axes of the projected ellipses Sigma' = [[a, b], [b, c]] (cov2d rows a, b, c; det > 0): sqrt(l1) v1
    and sqrt(l2) v2 with l1 >= l2 the eigenvalues, v1 the unit eigenvector of l1 taken from (l1 - c, b) when
    a >= c and else from (b, l1 - a), and v2 = v1 turned by +90 degrees (the axes Sec. 3.2 stores in fp16).
    Returns [4, n]: axis1.x, axis1.y, axis2.x, axis2.y."""
    a, b, c = (np.asarray(x, np.float64) for x in cov2d)
    det = a * c - b * b
    hd = 0.5 * (a - c)
    l1 = 0.5 * (a + c) + np.sqrt(hd * hd + b * b)
    l2 = det / l1
    vx = np.where(a >= c, l1 - c, b)
    vy = np.where(a >= c, b, l1 - a)
    nv = np.sqrt(vx * vx + vy * vy)
    safe = nv > 0
    vx = np.where(safe, vx / np.where(safe, nv, 1.0), 1.0)
    vy = np.where(safe, vy / np.where(safe, nv, 1.0), 0.0)
    s1, s2 = np.sqrt(l1), np.sqrt(l2)
    return np.stack([s1 * vx, s1 * vy, -s2 * vy, s2 * vx])


def pack_quantise(proj):
    """Sec. 3.2's packed render inputs, as the renderer then sees them: the ellipse axes rounded to IEEE fp16
    (nearest even), the ellipse rebuilt as axis1 axis1^T + axis2 axis2^T (determinant: the squared cross product
    of the axes) and inverted into the conic; colour clamped to [0, 1] and opacity, each stored as
    floor(255 x + 1/2) / 255 (RGBA8).  Returns (conic [3, n], opacity [n], rgb [3, n]) in fp64; rows of culled
    splats are left as they are."""
    vis = proj["status"] == 0
    cov = np.where(vis[None], proj["cov2d"], np.array([[1.0], [0.0], [1.0]]))
    ax = ellipse_axes(cov).astype(np.float16).astype(np.float64)
    a1x, a1y, a2x, a2y = ax
    s00, s01, s11 = a1x * a1x + a2x * a2x, a1x * a1y + a2x * a2y, a1y * a1y + a2y * a2y
    det = (a1x * a2y - a1y * a2x) ** 2
    conic = np.where(vis[None], np.stack([s11 / det, -s01 / det, s00 / det]), proj["conic"])
    q = lambda x: np.floor(255.0 * x + 0.5) / 255.0  # noqa: E731
    opacity = np.where(vis, q(np.asarray(proj["opacity"], np.float64)), proj["opacity"])
    rgb = np.where(vis[None], q(np.minimum(np.asarray(proj["rgb"], np.float64), 1.0)), proj["rgb"])
    return conic, opacity, rgb


def render(scene, cam, opts: Options, mode="tiled", mask=None, outcomes=False, packed=False) -> dict:
    """Whole forward path for one view.

    mode="tiled": preprocess, emit, stable sort, tile ranges, composite (the
    pipeline's own steps).  mode="brute": every validly projected Gaussian at
    every pixel in (fp32 depth bits, id) order, no culling (the definition).
    outcomes=True (tiled mode) attaches composite_outcomes() as out["outcomes"].
    packed=True (tiled mode) composites the packed render inputs of Sec. 3.2 (pack_quantise): the same pairs and
    pixel rectangles, the quantised ellipse, colour and opacity.
    """
    _check_opts(scene, opts)
    if mode == "brute":
        lib = _load()
        m, s, q, o, sh = _scene64(scene)
        out = _image_buffers(cam.height, cam.width)
        img = _Image(**{k: out[k].ctypes.data for k in out})
        mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        lib.orc_render_brute(scene.n, _dp(m), _dp(s), _dp(q), _dp(o), _dp(sh), C.byref(_cam(cam)),
                             C.byref(_opts(opts)), None if mk is None else mk.ctypes.data_as(C.POINTER(C.c_uint8)),
                             C.byref(img))
        return out
    proj = preprocess(scene, cam, opts)
    keys, vals = emit(scene, cam, opts)
    skeys, svals = stable_sort(keys, vals)
    tx, ty = tiles_xy(cam, opts)
    ranges = tile_ranges(skeys, tx * ty)
    conic, opacity, rgb = pack_quantise(proj) if packed else (proj["conic"], proj["opacity"], proj["rgb"])
    out = composite(proj["mean2d"], conic, opacity, rgb, proj["pix_rect"], cam, opts, svals, ranges, 0, mask,
                    outcomes=outcomes)
    out.update(proj=proj, keys=keys, vals=vals, sorted_keys=skeys, sorted_vals=svals, ranges=ranges)
    return out


def forward_backward(scene, cam, opts: Options, dL_dimage=None):
    """Forward of one view and, if dL_dimage [3,H,W] is given, its fp64 reverse mode.

    Returns dict(image, grads={means, log_scales, quats, opacity_logits, sh},
    splat_grad [n, 9] = dL/d(u, v, A, B, C, sigma, r, g, b), hash).
    """
    _check_opts(scene, opts)
    lib = _load()
    m, s, q, o, sh = _scene64(scene)
    n = scene.n
    H, W = cam.height, cam.width
    image = np.zeros((3, H, W))
    grads = dict(means=np.zeros((3, n)), log_scales=np.zeros((3, n)), quats=np.zeros((4, n)),
                 opacity_logits=np.zeros(n), sh=np.zeros_like(sh))
    splat_grad = np.zeros((n, 9))
    g = None if dL_dimage is None else _f64(dL_dimage)
    h = lib.orc_forward_backward(n, _dp(m), _dp(s), _dp(q), _dp(o), _dp(sh), C.byref(_cam(cam)),
                                 C.byref(_opts(opts)), None if g is None else _dp(g), _dp(image),
                                 _dp(grads["means"]), _dp(grads["log_scales"]), _dp(grads["quats"]),
                                 _dp(grads["opacity_logits"]), _dp(grads["sh"]), _dp(splat_grad))
    return dict(image=image, grads=grads, splat_grad=splat_grad, hash=int(h))


def set_threads(k: int) -> None:
    """Host threads of the oracle's loops over independent items (results do not depend on it)."""
    _load().orc_set_threads(int(k))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def sh_basis(direction, degree=3):
    lib = _load()
    d = _f64(direction)
    out = np.zeros(16)
    lib.orc_sh_basis(_dp(d), degree, _dp(out))
    return out[: (degree + 1) ** 2]


def quat_to_rotmat(q):
    lib = _load()
    qq = _f64(q)
    out = np.zeros(9)
    lib.orc_quat_to_rotmat(_dp(qq), _dp(out))
    return out.reshape(3, 3)


def l1_loss_grad(image, target):
    """Photometric L1 of the training workload (reading A19: the mean over every element of every view).

    `image` and `target` are arrays of the same shape, or equally long sequences of per-view arrays (views of
    any size).  Returns (loss, dL/dI): loss = sum |I - I*| / numel and dL/dI = sign(I - I*) / numel with
    sign(0) = 0, numel counting the elements of all views; the gradient comes back in the input's form.
    """
    views = isinstance(image, (list, tuple))
    imgs = list(image) if views else [image]
    tgts = list(target) if views else [target]
    if len(imgs) != len(tgts):
        raise ValueError("image and target hold different numbers of views")
    diffs = [np.asarray(i, np.float64) - np.asarray(t, np.float64) for i, t in zip(imgs, tgts)]
    numel = sum(d.size for d in diffs)
    loss = sum(float(np.abs(d).sum()) for d in diffs) / numel
    grads = [np.sign(d) / numel for d in diffs]
    return loss, (grads if views else grads[0])
