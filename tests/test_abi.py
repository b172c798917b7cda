"""The C-ABI library: it loads, exports every function the public header declares,
and its host-side entry points (sizes, validation, errors) behave as documented.
No call here enqueues GPU work, so the file runs without a GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2602_03207_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "websplat.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"#define[^\n]*", " ", text)
    names = set()
    for m in re.finditer(r"(?:^|;|\})\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(ws_\w+)\s*\(", text, flags=re.M):
        names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    return B.load()


def test_header_parses_to_the_expected_api():
    names = declared_functions()
    for core in ("ws_preprocess", "ws_sort", "ws_render", "ws_render_backward", "ws_last_error",
                 "ws_preprocess_workspace_size", "ws_sort_workspace_size", "ws_render_workspace_size",
                 "ws_render_backward_workspace_size"):
        assert core in names, core
    assert len(names) >= 20


def test_library_exports_every_declared_function(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = sorted(n for n in declared_functions() if n not in exported)
    assert not missing, missing
    for name in declared_functions():
        assert getattr(lib, name) is not None


def test_struct_layouts_match_the_header():
    assert C.sizeof(B.ws_camera) == 88 == B.CAMERA_BYTES
    assert B.ws_camera.R.offset == 24 and B.ws_camera.C.offset == 72
    assert C.sizeof(B.ws_options) == 64
    assert B.ws_options.bin_x.offset == 56 and B.ws_options.bin_y.offset == 60
    assert C.sizeof(B.ws_gaussians) == 48
    assert B.SPLAT_BYTES == 48


def test_binding_names_every_export_once():
    assert sorted(B.EXPORTED) == sorted(declared_functions())


def test_version_and_status_strings(lib):
    assert lib.ws_version() >= 100
    for s in range(0, 7):
        assert lib.ws_status_string(s)
    assert lib.ws_status_string(0).decode().lower().startswith("ok")


def _cam(w, h):
    c = B.ws_camera()
    c.width, c.height = w, h
    c.fx = c.fy = 100.0
    c.cx, c.cy = w / 2, h / 2
    for k in range(9):
        c.R[k] = 1.0 if k % 4 == 0 else 0.0
    return c


def _opts(**kw):
    o = B.make_options()
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def test_tile_and_image_counts(lib):
    cams = (B.ws_camera * 3)(_cam(1920, 1080), _cam(512, 512), _cam(77, 61))
    o = _opts(tile_w=16, tile_h=16)
    assert lib.ws_total_tiles(cams, 1, C.byref(o)) == 120 * 68
    assert lib.ws_total_tiles(cams, 3, C.byref(o)) == 120 * 68 + 32 * 32 + 5 * 4
    o8 = _opts(tile_w=8, tile_h=8)
    assert lib.ws_total_tiles(cams, 1, C.byref(o8)) == 240 * 135
    assert lib.ws_total_image_floats(cams, 3) == 3 * (1920 * 1080 + 512 * 512 + 77 * 61)


def test_workspace_sizes_are_monotone_and_aligned(lib):
    # small and large inputs use different sort schedules; sizes grow within each
    for caps in ((1, 1000, 1 << 20), ((1 << 20) + 1, 5_000_000, 50_000_000)):
        prev = 0
        for cap in caps:
            s = lib.ws_sort_workspace_size(cap, 32, 45, 8)
            assert s % 256 == 0 and s >= prev + 12 * (cap > 1), cap
            prev = s
    # one pass needs no ping-pong buffer; more passes do
    assert lib.ws_sort_workspace_size(1 << 22, 0, 8, 8) < lib.ws_sort_workspace_size(1 << 22, 0, 16, 8)
    assert lib.ws_preprocess_workspace_size(1000, 2, 10000, 8) >= lib.ws_preprocess_workspace_size(1000, 2, 10000, 0)
    assert lib.ws_render_backward_workspace_size(1000, 2) >= 9 * 1000 * 2 * 4
    assert lib.ws_l1_loss_workspace_size(1 << 20) > 0


def _err(lib):
    return lib.ws_last_error().decode()


def test_l1_loss_rejects_bad_arguments_on_the_host(lib):
    vp = C.c_void_p
    a, b, c, d, ws = vp(0x100000), vp(0x200000), vp(0x300000), vp(0x400000), vp(0x500000)
    need = lib.ws_l1_loss_workspace_size(100)
    # the batch's element count may not be below the call's
    st = lib.ws_l1_loss(a, b, 100, 99, c, d, ws, need, None)
    assert st == B.WS_ERR_INVALID_ARGUMENT and "total" in _err(lib)
    assert lib.ws_l1_loss(a, b, 100, -1, c, d, ws, need, None) == B.WS_ERR_INVALID_ARGUMENT
    assert lib.ws_l1_loss(a, b, 0, 0, c, d, ws, need, None) == B.WS_ERR_INVALID_ARGUMENT
    assert lib.ws_l1_loss(a, None, 100, 0, c, d, ws, need, None) == B.WS_ERR_INVALID_ARGUMENT
    assert lib.ws_l1_loss(a, b, 100, 0, c, d, ws, need - 1, None) == B.WS_ERR_WORKSPACE_TOO_SMALL


def test_backward_rejects_packed_records(lib):
    vp = C.c_void_p
    g = B.ws_gaussians()
    g.n = 10
    g.means = g.log_scales = g.quats = g.opacity_logits = g.sh = 0x100000
    grads = B.make_grads(0x200000, 0x200000, 0x200000, 0x200000, 0x200000)
    cams = (B.ws_camera * 1)(_cam(64, 64))
    o = _opts(flags=B.WS_FLAG_PACKED)
    st = lib.ws_render_backward(C.byref(g), cams, vp(0x300000), 1, C.byref(o), vp(0x400000), None, vp(0x500000),
                                vp(0x600000), vp(0x650000), vp(0x700000), vp(0x800000), C.byref(grads), vp(0x900000),
                                1 << 30, None)
    assert st == B.WS_ERR_UNSUPPORTED and "PACKED" in _err(lib)


def test_fused_l1_backward_rejects_bad_arguments_on_the_host(lib):
    vp = C.c_void_p
    g = B.ws_gaussians()
    g.n = 0
    grads = B.make_grads(0x200000, 0x200000, 0x200000, 0x200000, 0x200000)
    cams = (B.ws_camera * 2)(_cam(64, 48), _cam(32, 16))
    o = _opts()
    elems = 3 * (64 * 48 + 32 * 16)
    need = lib.ws_render_backward_l1_workspace_size(0, cams, 2, C.byref(o))
    # the per-tile loss sums come on top of the plain backward's workspace
    assert need >= lib.ws_render_backward_workspace_size(0, 2) + 8 * lib.ws_total_tiles(cams, 2, C.byref(o))
    assert lib.ws_render_backward_l1_workspace_size(-1, cams, 2, C.byref(o)) == 0

    def call(images=0x610000, targets=0x620000, total=0, loss=0x630000, ws_bytes=need):
        return lib.ws_render_backward_l1(C.byref(g), cams, vp(0x300000), 2, C.byref(o), vp(0x400000), None,
                                         vp(0x500000), vp(0x600000), vp(images) if images else None,
                                         vp(targets) if targets else None, total, vp(loss) if loss else None,
                                         vp(0x800000), C.byref(grads), vp(0x900000), ws_bytes, None)

    st = call(total=elems - 1)
    assert st == B.WS_ERR_INVALID_ARGUMENT and "total" in _err(lib)
    assert call(images=0) == B.WS_ERR_INVALID_ARGUMENT
    assert call(targets=0) == B.WS_ERR_INVALID_ARGUMENT
    assert call(loss=0) == B.WS_ERR_INVALID_ARGUMENT
    assert call(ws_bytes=need - 1) == B.WS_ERR_WORKSPACE_TOO_SMALL
    o.flags = B.WS_FLAG_PACKED
    assert call() == B.WS_ERR_UNSUPPORTED


def test_unknown_flags_are_rejected_and_accumulate_is_known(lib):
    vp = C.c_void_p
    g = B.ws_gaussians()
    g.n = 0
    cams = (B.ws_camera * 1)(_cam(64, 64))
    # the options pass validation with the accumulate flag: the call fails later, on the capacity
    o = _opts(flags=B.WS_FLAG_ACCUMULATE_GRADS)
    st = lib.ws_preprocess(C.byref(g), cams, vp(0x100000), 1, C.byref(o), None, None, None, None, -1,
                           vp(0x200000), vp(0x300000), vp(0x400000), 1 << 20, None)
    assert st == B.WS_ERR_INVALID_ARGUMENT and "capacity" in _err(lib)
    o.flags = 1 << 20
    st = lib.ws_preprocess(C.byref(g), cams, vp(0x100000), 1, C.byref(o), None, None, None, None, -1,
                           vp(0x200000), vp(0x300000), vp(0x400000), 1 << 20, None)
    assert st == B.WS_ERR_INVALID_ARGUMENT and "flag" in _err(lib)


def test_sort_rejects_bad_arguments_on_the_host(lib):
    vp = C.c_void_p
    a, b, c, d = vp(0x100000), vp(0x200000), vp(0x300000), vp(0x400000)
    ws = vp(0x500000)
    # begin >= end
    st = lib.ws_sort(a, b, c, d, 10, None, None, 20, 20, 8, ws, 1 << 20, None)
    assert st == B.WS_ERR_INVALID_ARGUMENT and "bit" in _err(lib)
    # end beyond 64
    assert lib.ws_sort(a, b, c, d, 10, None, None, 0, 65, 8, ws, 1 << 20, None) == B.WS_ERR_INVALID_ARGUMENT
    # radix width out of range
    assert lib.ws_sort(a, b, c, d, 10, None, None, 0, 32, 11, ws, 1 << 20, None) == B.WS_ERR_INVALID_ARGUMENT
    assert lib.ws_sort(a, b, c, d, 10, None, None, 0, 32, -1, ws, 1 << 20, None) == B.WS_ERR_INVALID_ARGUMENT
    assert lib.ws_sort_workspace_size(1000, 0, 32, 11) == 0 and lib.ws_sort_workspace_size(1000, 0, 32, 10) > 0
    # too many pairs
    assert lib.ws_sort(a, b, c, d, 1 << 30, None, None, 0, 32, 8, ws, 1 << 40, None) == B.WS_ERR_INVALID_ARGUMENT
    # output overlapping the input
    assert lib.ws_sort(a, b, a, d, 10, None, None, 0, 32, 8, ws, 1 << 20, None) == B.WS_ERR_INVALID_ARGUMENT
    # workspace too small / misaligned
    need = lib.ws_sort_workspace_size(1000, 0, 32, 8)
    assert lib.ws_sort(a, b, c, d, 1000, None, None, 0, 32, 8, ws, need - 1, None) == B.WS_ERR_WORKSPACE_TOO_SMALL
    assert lib.ws_sort(a, b, c, d, 1000, None, None, 0, 32, 8, vp(0x500004), need, None) == B.WS_ERR_INVALID_ARGUMENT


def test_sort32_rejects_bad_arguments_on_the_host(lib):
    vp = C.c_void_p
    a, b, c, d = vp(0x100000), vp(0x200000), vp(0x300000), vp(0x400000)
    ws = vp(0x500000)
    # bits beyond the 32-bit key
    st = lib.ws_sort32(a, b, c, d, 10, None, None, 0, 33, 8, ws, 1 << 20, None)
    assert st == B.WS_ERR_INVALID_ARGUMENT and "ws_sort32" in _err(lib) and "32" in _err(lib)
    assert lib.ws_sort32_workspace_size(1000, 0, 33, 8) == 0
    assert lib.ws_sort32(a, b, c, d, 10, None, None, 7, 7, 8, ws, 1 << 20, None) == B.WS_ERR_INVALID_ARGUMENT
    assert lib.ws_sort32(a, b, c, d, 10, None, None, 0, 32, 0, ws, 0, None) == B.WS_ERR_WORKSPACE_TOO_SMALL
    # keys of 4 bytes: outputs 4 * 10 bytes past the inputs do not overlap them, 4 * 10 - 1 do
    assert lib.ws_sort32(a, b, vp(0x100000 + 39), d, 10, None, None, 0, 32, 8, ws, 1 << 20, None) == \
        B.WS_ERR_INVALID_ARGUMENT
    need = lib.ws_sort32_workspace_size(10, 0, 32, 8)
    assert lib.ws_sort32(a, b, c, d, 0, None, None, 0, 32, 8, None, 0, None) == B.WS_OK
    assert lib.ws_sort32(a, b, c, d, 10, None, None, 0, 32, 8, ws, need - 1, None) == B.WS_ERR_WORKSPACE_TOO_SMALL
    # the 32-bit sort needs less workspace than the 64-bit one for the same pairs (half-width key buffer)
    assert lib.ws_sort32_workspace_size(1 << 20, 0, 32, 8) < lib.ws_sort_workspace_size(1 << 20, 0, 32, 8)


def test_preprocess_and_render_reject_bad_options_on_the_host(lib):
    g = B.ws_gaussians()
    g.n = 0
    cams = (B.ws_camera * 1)(_cam(64, 48))
    vp = C.c_void_p
    bad = [
        dict(tile_w=12, tile_h=12),
        dict(sh_degree=4),
        dict(radix_bits=11),
        dict(flags=1 << 12),
        dict(near_z=0.0),
        dict(alpha_min=0.0),
        dict(alpha_max=1.0),
        dict(t_min=0.0),
        dict(flags=B.WS_FLAG_KEYS32),  # 32-bit keys carry no depth: depth-first emission is required
    ]
    for kw in bad:
        o = _opts(**kw)
        st = lib.ws_preprocess(C.byref(g), cams, vp(0x1000), 1, C.byref(o), vp(0x2000), vp(0x3000), vp(0x4000),
                               vp(0x5000), 16, vp(0x6000), vp(0x7000), vp(0x8000), 1 << 20, None)
        assert st in (B.WS_ERR_INVALID_ARGUMENT, B.WS_ERR_UNSUPPORTED), kw
        assert _err(lib)
    o = _opts()
    bad_cam = (B.ws_camera * 1)(_cam(0, 48))
    st = lib.ws_render(vp(0x2000), 0, bad_cam, vp(0x1000), 1, C.byref(o), vp(0x4000), vp(0x5000), 16, vp(0x6000),
                       vp(0x7000), vp(0x9000), vp(0xa000), vp(0xb000), 1 << 20, None)
    assert st == B.WS_ERR_INVALID_ARGUMENT and "camera 0" in _err(lib)
    # n_views out of range, device cameras missing
    st = lib.ws_render(vp(0x2000), 0, cams, None, 1, C.byref(o), vp(0x4000), vp(0x5000), 16, vp(0x6000),
                       vp(0x7000), vp(0x9000), vp(0xa000), vp(0xb000), 1 << 20, None)
    assert st == B.WS_ERR_INVALID_ARGUMENT


def test_bin_counts_and_workspace(lib):
    cams = (B.ws_camera * 3)(_cam(1920, 1080), _cam(512, 512), _cam(77, 61))
    # 1x1 bins are tiles
    for tw, th in ((16, 16), (32, 16), (8, 8)):
        o = _opts(tile_w=tw, tile_h=th)
        assert lib.ws_total_bins(cams, 3, C.byref(o)) == lib.ws_total_tiles(cams, 3, C.byref(o))
        o.bin_x = o.bin_y = 0  # 0 reads as 1
        assert lib.ws_total_bins(cams, 3, C.byref(o)) == lib.ws_total_tiles(cams, 3, C.byref(o))
    # bins of 4x4 tiles of 32x16 pixels: 128x64-pixel cells, partial cells at the right / bottom edges
    o = _opts(tile_w=32, tile_h=16, bin_x=4, bin_y=4)
    want = sum(-(-w // 128) * -(-h // 64) for w, h in ((1920, 1080), (512, 512), (77, 61)))
    assert lib.ws_total_bins(cams, 3, C.byref(o)) == want == 15 * 17 + 4 * 8 + 1
    assert lib.ws_total_tiles(cams, 3, C.byref(o)) == 60 * 68 + 16 * 32 + 3 * 4
    o = _opts(tile_w=16, tile_h=8, bin_x=2, bin_y=8)
    assert lib.ws_total_bins(cams, 1, C.byref(o)) == 60 * 17
    assert lib.ws_expand_bins_workspace_size(cams, 3, C.byref(o)) >= 8 * lib.ws_total_bins(cams, 3, C.byref(o))


def test_bins_are_checked_on_the_host(lib):
    g = B.ws_gaussians()
    g.n = 0
    cams = (B.ws_camera * 1)(_cam(64, 48))
    vp = C.c_void_p
    for bx, by in ((3, 1), (1, 16), (-1, 1)):
        o = _opts(bin_x=bx, bin_y=by)
        st = lib.ws_preprocess(C.byref(g), cams, vp(0x1000), 1, C.byref(o), vp(0x2000), vp(0x3000), vp(0x4000),
                               vp(0x5000), 16, vp(0x6000), vp(0x7000), vp(0x8000), 1 << 20, None)
        assert st == B.WS_ERR_INVALID_ARGUMENT and "bin" in _err(lib), (bx, by)
    ws = vp(0x100000)
    # expansion needs bins larger than one tile
    o = _opts()
    st = lib.ws_expand_bins(vp(0x2000), 10, cams, vp(0x1000), 1, C.byref(o), vp(0x4000), vp(0x5000), 16,
                            vp(0x6000), vp(0x7000), vp(0x8000), 64, vp(0x9000), ws, 1 << 20, None)
    assert st == B.WS_ERR_INVALID_ARGUMENT and "bins" in _err(lib)
    # the tile lists need bin_x * bin_y slots per pair
    o = _opts(bin_x=2, bin_y=2)
    st = lib.ws_expand_bins(vp(0x2000), 10, cams, vp(0x1000), 1, C.byref(o), vp(0x4000), vp(0x5000), 16,
                            vp(0x6000), vp(0x7000), vp(0x8000), 63, vp(0x9000), ws, 1 << 20, None)
    assert st == B.WS_ERR_INVALID_ARGUMENT and "tile_capacity" in _err(lib)
    st = lib.ws_expand_bins(vp(0x2000), 10, cams, vp(0x1000), 1, C.byref(o), vp(0x4000), vp(0x5000), 1 << 30,
                            vp(0x6000), vp(0x7000), vp(0x8000), 1 << 32, vp(0x9000), ws, 1 << 20, None)
    assert st == B.WS_ERR_INVALID_ARGUMENT
    # workspace too small
    st = lib.ws_expand_bins(vp(0x2000), 10, cams, vp(0x1000), 1, C.byref(o), vp(0x4000), vp(0x5000), 16,
                            vp(0x6000), vp(0x7000), vp(0x8000), 64, vp(0x9000), ws, 0, None)
    assert st == B.WS_ERR_WORKSPACE_TOO_SMALL
    # with bins the render takes the expanded lists, never the bin keys
    st = lib.ws_render(vp(0x2000), 10, cams, vp(0x1000), 1, C.byref(o), vp(0x4000), vp(0x5000), 16, vp(0x6000),
                       vp(0x7000), vp(0x9000), vp(0xa000), vp(0xb000), 1 << 20, None)
    assert st == B.WS_ERR_INVALID_ARGUMENT and "ws_expand_bins" in _err(lib)


def test_product_path_fails_loudly_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        B.load()
