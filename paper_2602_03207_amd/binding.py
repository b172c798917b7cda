"""ctypes binding of libwebsplat (the C ABI declared in include/websplat.h).

Argument marshalling only: every function below converts torch tensors (device
memory) and Python values into the C types of the same-named C function, calls
it, and raises WsError on a non-OK status.  No arithmetic of the render path
happens here.  If the library has not been built, loading raises instead of
falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwebsplat.so")

WS_OK = 0
WS_ERR_INVALID_ARGUMENT = 1
WS_ERR_UNSUPPORTED = 2
WS_ERR_WORKSPACE_TOO_SMALL = 3
WS_ERR_HIP = 4
WS_ERR_CAPACITY = 5
WS_ERR_SPIN_LIMIT = 6

WS_FLAG_FIXED_3SIGMA = 1
WS_FLAG_NO_VIEWPORT_CULL = 2
WS_FLAG_ORDERED_RENDER = 4
WS_FLAG_DEPTH_FIRST = 8
WS_FLAG_KEYS32 = 16
WS_FLAG_ACCUMULATE_GRADS = 32
WS_FLAG_PACKED = 64

EXPORTED = [
    "ws_preprocess_workspace_size", "ws_sort_workspace_size", "ws_render_workspace_size",
    "ws_render_backward_workspace_size", "ws_total_tiles", "ws_total_image_floats", "ws_preprocess", "ws_sort",
    "ws_render", "ws_render_backward", "ws_l1_loss", "ws_l1_loss_workspace_size", "ws_graph_begin", "ws_graph_end",
    "ws_graph_launch", "ws_graph_destroy", "ws_last_error", "ws_status_string", "ws_version", "ws_timing_start",
    "ws_timing_stop", "ws_total_bins", "ws_expand_bins_workspace_size", "ws_expand_bins", "ws_sort32",
    "ws_sort32_workspace_size", "ws_sort_noalloc", "ws_render_backward_l1", "ws_render_backward_l1_workspace_size",
]

KERNELS = {"preprocess": 0, "scan_emit": 1, "sort_hist": 2, "sort_pass": 3, "ranges": 4, "render": 5,
           "render_bwd": 6, "preprocess_bwd": 7}


class WsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"websplat status {status}: {message}")
        self.status = status


class ws_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("C", C.c_float * 3), ("reserved", C.c_int32)]


class ws_options(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("sh_degree", C.c_int32), ("radix_bits", C.c_int32),
                ("flags", C.c_uint32), ("near_z", C.c_float), ("lowpass", C.c_float), ("clamp_fov", C.c_float),
                ("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float), ("bg", C.c_float * 3),
                ("bin_x", C.c_int32), ("bin_y", C.c_int32)]


class ws_gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p)]


class ws_gaussian_grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p)]


SPLAT_BYTES = 48
PACKED_SPLAT_BYTES = 32
CAMERA_BYTES = C.sizeof(ws_camera)

_lib = None


def load():
    """Load libwebsplat.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run paper_2602_03207_amd.build.build() "
                           "(or __graft_entry__.build()) first")
    lib = C.CDLL(LIB_PATH)
    P, vp, i64, i32, sz = C.POINTER, C.c_void_p, C.c_int64, C.c_int32, C.c_size_t
    lib.ws_preprocess_workspace_size.argtypes = [i64, i32, i64, C.c_uint32]
    lib.ws_preprocess_workspace_size.restype = sz
    lib.ws_sort_workspace_size.argtypes = [i64, i32, i32, i32]
    lib.ws_sort_workspace_size.restype = sz
    lib.ws_sort32_workspace_size.argtypes = [i64, i32, i32, i32]
    lib.ws_sort32_workspace_size.restype = sz
    lib.ws_render_workspace_size.argtypes = [P(ws_camera), i32, P(ws_options)]
    lib.ws_render_workspace_size.restype = sz
    lib.ws_render_backward_workspace_size.argtypes = [i64, i32]
    lib.ws_render_backward_workspace_size.restype = sz
    lib.ws_l1_loss_workspace_size.argtypes = [i64]
    lib.ws_l1_loss_workspace_size.restype = sz
    lib.ws_total_tiles.argtypes = [P(ws_camera), i32, P(ws_options)]
    lib.ws_total_tiles.restype = i64
    lib.ws_total_bins.argtypes = [P(ws_camera), i32, P(ws_options)]
    lib.ws_total_bins.restype = i64
    lib.ws_expand_bins_workspace_size.argtypes = [P(ws_camera), i32, P(ws_options)]
    lib.ws_expand_bins_workspace_size.restype = sz
    lib.ws_expand_bins.argtypes = [vp, i64, P(ws_camera), vp, i32, P(ws_options), vp, vp, i64, vp, vp, vp, i64, vp,
                                   vp, sz, vp]
    lib.ws_total_image_floats.argtypes = [P(ws_camera), i32]
    lib.ws_total_image_floats.restype = i64
    lib.ws_preprocess.argtypes = [P(ws_gaussians), P(ws_camera), vp, i32, P(ws_options), vp, vp, vp, vp, i64, vp,
                                  vp, vp, sz, vp]
    lib.ws_sort.argtypes = [vp, vp, vp, vp, i64, vp, vp, i32, i32, i32, vp, sz, vp]
    lib.ws_sort32.argtypes = [vp, vp, vp, vp, i64, vp, vp, i32, i32, i32, vp, sz, vp]
    lib.ws_sort_noalloc.argtypes = [vp, vp, vp, vp, i64, vp, vp, i32, i32, i32, vp]
    lib.ws_render.argtypes = [vp, i64, P(ws_camera), vp, i32, P(ws_options), vp, vp, i64, vp, vp, vp, vp, vp, sz,
                              vp]
    lib.ws_render_backward.argtypes = [P(ws_gaussians), P(ws_camera), vp, i32, P(ws_options), vp, vp, vp, vp, vp,
                                       vp, vp, P(ws_gaussian_grads), vp, sz, vp]
    lib.ws_render_backward_l1.argtypes = [P(ws_gaussians), P(ws_camera), vp, i32, P(ws_options), vp, vp, vp, vp, vp,
                                          vp, i64, vp, vp, P(ws_gaussian_grads), vp, sz, vp]
    lib.ws_render_backward_l1_workspace_size.argtypes = [i64, P(ws_camera), i32, P(ws_options)]
    lib.ws_render_backward_l1_workspace_size.restype = sz
    lib.ws_l1_loss.argtypes = [vp, vp, i64, i64, vp, vp, vp, sz, vp]
    lib.ws_graph_begin.argtypes = [vp]
    lib.ws_graph_end.argtypes = [vp, P(vp)]
    lib.ws_graph_launch.argtypes = [vp, vp]
    lib.ws_graph_destroy.argtypes = [vp]
    lib.ws_last_error.restype = C.c_char_p
    lib.ws_status_string.argtypes = [i32]
    lib.ws_status_string.restype = C.c_char_p
    lib.ws_version.restype = i32
    lib.ws_timing_start.argtypes = [i32]
    lib.ws_timing_stop.argtypes = [P(C.c_double), P(C.c_int64)]
    for name in ("ws_timing_start", "ws_timing_stop", "ws_preprocess", "ws_sort", "ws_sort32", "ws_sort_noalloc",
                 "ws_expand_bins",
                 "ws_render",
                 "ws_render_backward", "ws_l1_loss", "ws_graph_begin",
                 "ws_graph_end", "ws_graph_launch", "ws_graph_destroy"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(status):
    if status != WS_OK:
        lib = load()
        raise WsError(status, lib.ws_last_error().decode(errors="replace"))


def _ptr(t):
    """Device (or host) address of a tensor / ndarray, None for None."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------ struct builders

def make_camera(cam) -> ws_camera:
    """ws_camera from any object with width, height, fx, fy, cx, cy, R (3x3), t (3), C (3)."""
    c = ws_camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.R[:] = [float(x) for x in np.asarray(cam.R, np.float32).reshape(9)]
    c.t[:] = [float(x) for x in np.asarray(cam.t, np.float32).reshape(3)]
    c.C[:] = [float(x) for x in np.asarray(cam.C, np.float32).reshape(3)]
    c.reserved = 0
    return c


def camera_array(cams):
    arr = (ws_camera * len(cams))()
    for i, cam in enumerate(cams):
        arr[i] = make_camera(cam)
    return arr


def camera_bytes(cam_arr) -> np.ndarray:
    """Raw bytes of a ws_camera array (to upload as the device copy)."""
    return np.frombuffer(bytes(cam_arr), dtype=np.uint8).copy()


def make_options(tile_w=16, tile_h=16, sh_degree=0, radix_bits=0, flags=0, near_z=0.2, lowpass=0.3, clamp_fov=1.3,
                 alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, bg=(0.0, 0.0, 0.0), bin_x=1, bin_y=1) -> ws_options:
    o = ws_options()
    o.tile_w, o.tile_h, o.sh_degree, o.radix_bits, o.flags = tile_w, tile_h, sh_degree, radix_bits, flags
    o.bin_x, o.bin_y = bin_x, bin_y
    o.near_z, o.lowpass, o.clamp_fov = near_z, lowpass, clamp_fov
    o.alpha_min, o.alpha_max, o.t_min = alpha_min, alpha_max, t_min
    o.bg[:] = [float(b) for b in bg]
    return o


def make_gaussians(n, means, log_scales, quats, opacity_logits, sh) -> ws_gaussians:
    g = ws_gaussians()
    g.n = int(n)
    g.means, g.log_scales, g.quats = _ptr(means), _ptr(log_scales), _ptr(quats)
    g.opacity_logits, g.sh = _ptr(opacity_logits), _ptr(sh)
    return g


def make_grads(means, log_scales, quats, opacity_logits, sh) -> ws_gaussian_grads:
    g = ws_gaussian_grads()
    g.means, g.log_scales, g.quats = _ptr(means), _ptr(log_scales), _ptr(quats)
    g.opacity_logits, g.sh = _ptr(opacity_logits), _ptr(sh)
    return g


# -------------------------------------------------------------------- sizes

def ws_preprocess_workspace_size(n, n_views, capacity, flags=0):
    return load().ws_preprocess_workspace_size(n, n_views, capacity, flags)


def ws_sort_workspace_size(capacity, begin_bit, end_bit, radix_bits=0):
    return load().ws_sort_workspace_size(capacity, begin_bit, end_bit, radix_bits)


def ws_sort32_workspace_size(capacity, begin_bit, end_bit, radix_bits=0):
    return load().ws_sort32_workspace_size(capacity, begin_bit, end_bit, radix_bits)


def ws_render_workspace_size(cams, n_views, opt):
    return load().ws_render_workspace_size(cams, n_views, C.byref(opt))


def ws_render_backward_workspace_size(n, n_views):
    return load().ws_render_backward_workspace_size(n, n_views)


def ws_render_backward_l1_workspace_size(n, cams, n_views, opt):
    return load().ws_render_backward_l1_workspace_size(n, cams, n_views, C.byref(opt))


def ws_l1_loss_workspace_size(n):
    return load().ws_l1_loss_workspace_size(n)


def ws_total_tiles(cams, n_views, opt):
    return load().ws_total_tiles(cams, n_views, C.byref(opt))


def ws_total_bins(cams, n_views, opt):
    return load().ws_total_bins(cams, n_views, C.byref(opt))


def ws_expand_bins_workspace_size(cams, n_views, opt):
    return load().ws_expand_bins_workspace_size(cams, n_views, C.byref(opt))


def ws_total_image_floats(cams, n_views):
    return load().ws_total_image_floats(cams, n_views)


# ---------------------------------------------------------------- the path

def ws_preprocess(g, cams, d_cams, n_views, opt, splats, tiles_touched, keys, values, capacity, d_num_pairs,
                  d_status, ws, ws_bytes, stream=None):
    _check(load().ws_preprocess(C.byref(g), cams, _ptr(d_cams), n_views, C.byref(opt), _ptr(splats),
                                _ptr(tiles_touched), _ptr(keys), _ptr(values), capacity, _ptr(d_num_pairs),
                                _ptr(d_status), _ptr(ws), ws_bytes, _stream(stream)))


def ws_sort(keys_in, values_in, keys_out, values_out, n, d_n, d_status, begin_bit, end_bit, radix_bits, ws,
            ws_bytes, stream=None):
    _check(load().ws_sort(_ptr(keys_in), _ptr(values_in), _ptr(keys_out), _ptr(values_out), n, _ptr(d_n),
                          _ptr(d_status), begin_bit, end_bit, radix_bits, _ptr(ws), ws_bytes, _stream(stream)))


def ws_sort32(keys_in, values_in, keys_out, values_out, n, d_n, d_status, begin_bit, end_bit, radix_bits, ws,
              ws_bytes, stream=None):
    _check(load().ws_sort32(_ptr(keys_in), _ptr(values_in), _ptr(keys_out), _ptr(values_out), n, _ptr(d_n),
                            _ptr(d_status), begin_bit, end_bit, radix_bits, _ptr(ws), ws_bytes, _stream(stream)))


def ws_sort_noalloc(keys_in, values_in, keys_out, values_out, n, d_n, d_status, begin_bit, end_bit, radix_bits,
                    stream=None):
    _check(load().ws_sort_noalloc(_ptr(keys_in), _ptr(values_in), _ptr(keys_out), _ptr(values_out), n, _ptr(d_n),
                                  _ptr(d_status), begin_bit, end_bit, radix_bits, _stream(stream)))


def ws_expand_bins(splats, n, cams, d_cams, n_views, opt, keys, values, capacity, d_num_pairs, d_status, tile_values,
                   tile_capacity, tile_ranges, ws, ws_bytes, stream=None):
    _check(load().ws_expand_bins(_ptr(splats), n, cams, _ptr(d_cams), n_views, C.byref(opt), _ptr(keys),
                                 _ptr(values), capacity, _ptr(d_num_pairs), _ptr(d_status), _ptr(tile_values),
                                 tile_capacity, _ptr(tile_ranges), _ptr(ws), ws_bytes, _stream(stream)))


def ws_render(splats, n, cams, d_cams, n_views, opt, keys, values, capacity, d_num_pairs, d_status, tile_ranges,
              images, ws, ws_bytes, stream=None):
    _check(load().ws_render(_ptr(splats), n, cams, _ptr(d_cams), n_views, C.byref(opt), _ptr(keys), _ptr(values),
                            capacity, _ptr(d_num_pairs), _ptr(d_status), _ptr(tile_ranges), _ptr(images), _ptr(ws),
                            ws_bytes, _stream(stream)))


def ws_render_backward(g, cams, d_cams, n_views, opt, splats, tiles_touched, values, tile_ranges, images,
                       dL_dimages, d_status, grads, ws, ws_bytes, stream=None):
    _check(load().ws_render_backward(C.byref(g), cams, _ptr(d_cams), n_views, C.byref(opt), _ptr(splats),
                                     _ptr(tiles_touched), _ptr(values), _ptr(tile_ranges), _ptr(images), _ptr(dL_dimages), _ptr(d_status),
                                     C.byref(grads), _ptr(ws), ws_bytes, _stream(stream)))


def ws_render_backward_l1(g, cams, d_cams, n_views, opt, splats, tiles_touched, values, tile_ranges, images,
                          targets, total, d_loss, d_status, grads, ws, ws_bytes, stream=None):
    _check(load().ws_render_backward_l1(C.byref(g), cams, _ptr(d_cams), n_views, C.byref(opt), _ptr(splats),
                                        _ptr(tiles_touched), _ptr(values), _ptr(tile_ranges), _ptr(images), _ptr(targets), total,
                                        _ptr(d_loss), _ptr(d_status), C.byref(grads), _ptr(ws), ws_bytes,
                                        _stream(stream)))


def ws_l1_loss(images, targets, n, total, dL_dimages, d_loss, ws, ws_bytes, stream=None):
    _check(load().ws_l1_loss(_ptr(images), _ptr(targets), n, total, _ptr(dL_dimages), _ptr(d_loss), _ptr(ws),
                             ws_bytes, _stream(stream)))


def ws_graph_begin(stream):
    _check(load().ws_graph_begin(_stream(stream)))


def ws_graph_end(stream):
    out = C.c_void_p()
    _check(load().ws_graph_end(_stream(stream), C.byref(out)))
    return out.value


def ws_graph_launch(graph, stream):
    _check(load().ws_graph_launch(graph, _stream(stream)))


def ws_graph_destroy(graph):
    _check(load().ws_graph_destroy(graph))


def ws_last_error():
    return load().ws_last_error().decode(errors="replace")


def ws_status_string(status):
    return load().ws_status_string(status).decode()


def ws_version():
    return load().ws_version()


def ws_timing_start(kernel):
    _check(load().ws_timing_start(KERNELS[kernel] if isinstance(kernel, str) else kernel))


def ws_timing_stop():
    """Returns (summed milliseconds, launches) of the kernel being timed."""
    ms = C.c_double()
    n = C.c_int64()
    _check(load().ws_timing_stop(C.byref(ms), C.byref(n)))
    return ms.value, n.value
