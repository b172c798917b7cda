"""ws_render on the GPU: per-component and end-to-end image parity with the oracle, and invariances."""
import numpy as np
import pytest

import oracle
import scenegen
from _helpers import assert_image_parity, gpu_options, oracle_options, pack_splats

pytestmark = pytest.mark.gpu


def _full(scene, cams, **kw):
    import torch
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    r = Renderer(cams, gpu_options(sh_degree=scene.sh_degree, **kw))
    r.forward(GaussianTensors.from_scene(scene))
    torch.cuda.synchronize()
    return r


def _check_ranges(rg, ref_ranges, sorted_keys):
    """Non-empty tile ranges equal the oracle's; an empty tile's range is empty.  Every range is
    [first pair with tile >= t, first pair with tile > t) of the sorted key list."""
    ref_ranges = np.asarray(ref_ranges, np.int64)
    full = ref_ranges[:, 1] > ref_ranges[:, 0]
    assert np.array_equal(rg[full], ref_ranges[full])
    assert np.all(rg[~full, 0] == rg[~full, 1])
    tiles = (np.asarray(sorted_keys, np.uint64) >> np.uint64(32)).astype(np.int64)
    t = np.arange(rg.shape[0])
    assert np.array_equal(rg[:, 0], np.searchsorted(tiles, t, "left"))
    assert np.array_equal(rg[:, 1], np.searchsorted(tiles, t, "right"))


def _ranges_of(keys_np, n_tiles, width, height, tile=16):
    """ws_render's tile ranges for a given sorted key list (invisible splats, so only the ranges matter)."""
    import torch
    from paper_2602_03207_amd import binding as B
    m = keys_np.size
    opts = gpu_options(tile_w=tile, tile_h=tile)
    cam = scenegen.Camera(width, height, 500.0, 500.0, width / 2, height / 2, np.eye(3), np.zeros(3), np.zeros(3))
    cams = B.camera_array([cam])
    assert B.ws_total_tiles(cams, 1, opts) == n_tiles
    d_cams = torch.as_tensor(B.camera_bytes(cams)).cuda()
    rec = np.zeros((4, 12), np.float32)  # zero opacity, empty rectangles
    splats = torch.as_tensor(rec).cuda()
    keys = torch.as_tensor(keys_np.view(np.int64)).cuda() if m else torch.zeros(1, dtype=torch.int64, device="cuda")
    vals = torch.zeros(max(m, 1), dtype=torch.int32, device="cuda")
    d_n = torch.tensor([m], dtype=torch.int64, device="cuda")
    d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ranges = torch.full((2 * n_tiles,), 0x7f7f7f7f, dtype=torch.int32, device="cuda")
    images = torch.empty(3 * width * height, dtype=torch.float32, device="cuda")
    ws = torch.empty(max(B.ws_render_workspace_size(cams, 1, opts), 256), dtype=torch.uint8, device="cuda")
    B.ws_render(splats, 4, cams, d_cams, 1, opts, keys, vals, max(m, 1), d_n, d_status, ranges, images, ws,
                ws.numel())
    torch.cuda.synchronize()
    assert int(d_status.item()) == 0
    return ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)


def test_tile_ranges_cover_every_tile():
    """Every tile's range is written whatever the gaps: none before the first run, long gaps (more than a
    wave and a workgroup of empty tiles), runs longer than a chunk, keys past the last tile, no keys at all."""
    W, H = 1000, 600
    T = 63 * 38
    rng = np.random.default_rng(11)
    cases = [
        np.array([], np.int64),
        np.array([5] * 3 + [6] + [400] * 2 + [401] + [2000] * 5000 + [T - 2], np.int64),
        np.array([0] + [1] * 70 + [T - 1] * 3 + [T, T, T + 9], np.int64),
        np.sort(rng.choice(T, 300, replace=False).repeat(rng.integers(1, 40, 300))),
        np.full(20000, 17, np.int64),
    ]
    for tiles in cases:
        keys = (tiles.astype(np.uint64) << np.uint64(32)) | rng.integers(0, 1 << 31, tiles.size).astype(np.uint64)
        rg = _ranges_of(keys, T, W, H)
        t = np.arange(T)
        assert np.array_equal(rg[:, 0], np.searchsorted(tiles, t, "left")), tiles[:10]
        assert np.array_equal(rg[:, 1], np.searchsorted(tiles, t, "right")), tiles[:10]


def test_render_component_parity_c1():
    """Render fed the oracle's fp32-rounded splats and sorted pairs vs the oracle compositing them."""
    import torch
    from paper_2602_03207_amd import binding as B
    scene, cam = scenegen.c1()
    ro = oracle_options()
    ref = oracle.render(scene, cam, ro)
    p = ref["proj"]
    vis = p["status"] == 0
    f32 = lambda a: np.asarray(a, np.float32)  # noqa: E731
    rec = pack_splats(f32(p["mean2d"]), f32(p["conic"]), f32(p["opacity"]), f32(p["rgb"]), p["depth32"],
                      np.where(vis, p["pix_rect"], 0))
    comp = oracle.composite(f32(p["mean2d"]), f32(p["conic"]), f32(p["opacity"]), f32(p["rgb"]), p["pix_rect"], cam,
                            ro, ref["sorted_vals"], ref["ranges"], outcomes=True)
    m = ref["sorted_keys"].size
    opts = gpu_options()
    cams = B.camera_array([cam])
    d_cams = torch.as_tensor(B.camera_bytes(cams)).cuda()
    splats = torch.as_tensor(rec).cuda()
    keys = torch.as_tensor(ref["sorted_keys"].view(np.int64)).cuda()
    vals = torch.as_tensor(ref["sorted_vals"].view(np.int32)).cuda()
    d_n = torch.tensor([m], dtype=torch.int64, device="cuda")
    d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
    tiles = B.ws_total_tiles(cams, 1, opts)
    ranges = torch.empty(2 * tiles, dtype=torch.int32, device="cuda")
    images = torch.empty(3 * cam.width * cam.height, dtype=torch.float32, device="cuda")
    ws = torch.empty(max(B.ws_render_workspace_size(cams, 1, opts), 256), dtype=torch.uint8, device="cuda")
    B.ws_render(splats, scene.n, cams, d_cams, 1, opts, keys, vals, m, d_n, d_status, ranges, images, ws, ws.numel())
    torch.cuda.synchronize()
    rg = ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    _check_ranges(rg, ref["ranges"], ref["sorted_keys"])
    img = images.cpu().numpy().reshape(3, cam.height, cam.width)
    worst, frac = assert_image_parity(img, comp)
    assert worst < 2e-5


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 16)])
def test_quadrant_culling_keeps_every_contribution(tile):
    """Thin, rotated, faint and large splats (the cases where a splat's rectangle holds quadrants its
    alpha >= alpha_min ellipse never reaches) rendered from given records and pairs: every pixel matches
    the oracle compositing the same records, so the quadrant culling drops no contributing splat."""
    import torch
    from paper_2602_03207_amd import binding as B
    tw, th = tile
    W, H, n = 512, 384, 3000
    rng = np.random.default_rng(23)
    u, v = rng.uniform(-30, W + 30, n), rng.uniform(-30, H + 30, n)
    s1 = np.exp(rng.uniform(np.log(0.5), np.log(90), n))
    s2 = s1 / np.exp(rng.uniform(0, np.log(300), n))
    th_ = rng.uniform(0, np.pi, n)
    c, s_ = np.cos(th_), np.sin(th_)
    S00 = c * c * s1 * s1 + s_ * s_ * s2 * s2 + 0.3
    S11 = s_ * s_ * s1 * s1 + c * c * s2 * s2 + 0.3
    S01 = c * s_ * (s1 * s1 - s2 * s2)
    det = S00 * S11 - S01 * S01
    conic = np.stack([S11 / det, -S01 / det, S00 / det]).astype(np.float32)
    opacity = np.exp(rng.uniform(np.log(1.02 / 255), np.log(0.99), n)).astype(np.float32)
    rgb = rng.uniform(0.2, 1.0, (3, n)).astype(np.float32)
    depth = rng.permutation(np.linspace(1.0, 50.0, n)).astype(np.float32)
    mean2d = np.stack([u, v]).astype(np.float32)
    d2 = 2 * np.log(255 * opacity.astype(np.float64))
    hx, hy = np.sqrt(d2 * S00), np.sqrt(d2 * S11)
    rect = np.stack([np.ceil(u - hx - 0.5), np.floor(u + hx - 0.5), np.ceil(v - hy - 0.5), np.floor(v + hy - 0.5)])
    rect = np.stack([np.clip(rect[0], 0, W - 1), np.clip(rect[1], -1, W - 1), np.clip(rect[2], 0, H - 1),
                     np.clip(rect[3], -1, H - 1)]).astype(np.int32)
    vis = (rect[1] >= rect[0]) & (rect[3] >= rect[2]) & (u - hx < W) & (u + hx > 0) & (v - hy < H) & (v + hy > 0)
    tx = (W + tw - 1) // tw
    keys, vals = [], []
    for i in np.nonzero(vis)[0]:
        for ty in range(rect[2, i] // th, rect[3, i] // th + 1):
            for t in range(rect[0, i] // tw, rect[1, i] // tw + 1):
                keys.append((ty * tx + t) << 32 | int(depth[i:i + 1].view(np.uint32)[0]))
                vals.append(i)
    keys, vals = np.array(keys, np.uint64), np.array(vals, np.uint32)
    skeys, svals = oracle.stable_sort(keys, vals)
    n_tiles = tx * ((H + th - 1) // th)
    ranges = oracle.tile_ranges(skeys, n_tiles)
    cam = scenegen.Camera(W, H, 400.0, 400.0, W / 2, H / 2, np.eye(3), np.zeros(3), np.zeros(3))
    ro = oracle_options(tile_w=tw, tile_h=th)
    rect_or = np.where(vis, rect, np.array([[1], [0], [1], [0]], np.int32))
    comp = oracle.composite(mean2d, conic, opacity, rgb, rect_or, cam, ro, svals, ranges, outcomes=True)
    rec = pack_splats(mean2d, conic, opacity, rgb, depth, np.where(vis, rect, 0))
    opts = gpu_options(tile_w=tw, tile_h=th)
    cams = B.camera_array([cam])
    d_cams = torch.as_tensor(B.camera_bytes(cams)).cuda()
    m = skeys.size
    d_n = torch.tensor([m], dtype=torch.int64, device="cuda")
    d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ranges_d = torch.empty(2 * n_tiles, dtype=torch.int32, device="cuda")
    images = torch.empty(3 * W * H, dtype=torch.float32, device="cuda")
    ws = torch.empty(max(B.ws_render_workspace_size(cams, 1, opts), 256), dtype=torch.uint8, device="cuda")
    B.ws_render(torch.as_tensor(rec).cuda(), n, cams, d_cams, 1, opts, torch.as_tensor(skeys.view(np.int64)).cuda(),
                torch.as_tensor(svals.view(np.int32)).cuda(), m, d_n, d_status, ranges_d, images, ws, ws.numel())
    torch.cuda.synchronize()
    assert int(d_status.item()) == 0
    img = images.cpu().numpy().reshape(3, H, W)
    assert_image_parity(img, comp)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 8), (32, 16)])
def test_render_end_to_end_c1(tile):
    scene, cam = scenegen.c1()
    r = _full(scene, [cam], tile_w=tile[0], tile_h=tile[1])
    ref = oracle.render(scene, cam, oracle_options(*tile), outcomes=True)
    assert r.num_pairs == ref["keys"].size
    assert_image_parity(r.image(0).cpu().numpy(), ref)


def test_render_end_to_end_tiny_near_plane_sh2():
    scene = scenegen.random_scene(3000, 21, mean_lo=-1.5, mean_hi=1.5, log_scale_mu=-2.8, log_scale_sd=0.6,
                                  logit_sd=2.5, sh_degree=2, dc_sd=0.5, rest_sd=0.2)
    cam = scenegen.look_at([0.2, 0.1, -0.6], [0, 0, 1], 161, 97)  # ragged tiles in both directions
    r = _full(scene, [cam])
    ref = oracle.render(scene, cam, oracle_options(sh_degree=2), outcomes=True)
    assert_image_parity(r.image(0).cpu().numpy(), ref)


def test_render_background_and_empty_scene():
    scene = scenegen.random_scene(0, 1)
    cam = scenegen.look_at([0, 0, -3], [0, 0, 0], 40, 24)
    r = _full(scene, [cam], bg=(0.25, 0.5, 1.0))
    img = r.image(0).cpu().numpy()
    assert r.num_pairs == 0
    for ch, b in enumerate((0.25, 0.5, 1.0)):
        assert np.all(img[ch] == np.float32(b))
    # every Gaussian culled (behind the camera)
    scene = scenegen.random_scene(500, 2)
    scene.means[2] = np.float32(-10.0)
    r = _full(scene, [cam])
    assert r.num_pairs == 0 and np.all(r.image(0).cpu().numpy() == 0)


@pytest.mark.slow
@pytest.mark.parametrize("depth_first", [False, True])
def test_render_end_to_end_c2(depth_first):
    from paper_2602_03207_amd import binding as B
    scene, cam = scenegen.c2()
    r = _full(scene, [cam], flags=B.WS_FLAG_DEPTH_FIRST if depth_first else 0)
    ref = oracle.render(scene, cam, oracle_options(sh_degree=3), outcomes=True)
    worst, frac = assert_image_parity(r.image(0).cpu().numpy(), ref)
    print(f"C2: worst {worst:.2e}, flagged {frac:.2e}, M gpu {r.num_pairs} oracle {ref['keys'].size}")


@pytest.mark.slow
def test_render_c2_in_the_benchmark_configuration():
    """The headline frame exactly as bench.py times it (depth-first emission, 32-bit tile keys, one graph
    replay of the device-sized forward) in the layouts its autotuner picks among (16x16 tiles in 2x2 or 4x2
    bins, 32x16 tiles without bins), each against the oracle's image of the same view."""
    import torch
    from paper_2602_03207_amd import binding as B
    from paper_2602_03207_amd.batched import BatchedForward
    from paper_2602_03207_amd.pipeline import GaussianTensors
    scene, cam = scenegen.c2()
    g = GaussianTensors.from_scene(scene)
    ref = oracle.render(scene, cam, oracle_options(sh_degree=3), outcomes=True)
    flags = B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32
    for tile, bins, rb in (((16, 16), (4, 2), 9), ((16, 16), (2, 2), 6), ((32, 16), (4, 4), 8), ((32, 16), (1, 1), 6)):
        print(f"C2 benchmark layout: tile {tile} bins {bins} radix {rb}", flush=True)
        opts = gpu_options(sh_degree=3, tile_w=tile[0], tile_h=tile[1], radix_bits=rb, flags=flags, bin_x=bins[0],
                           bin_y=bins[1])
        bf = BatchedForward([cam], opts, g)
        bf.capture()
        for _ in range(3):
            bf.replay()
        bf.check()
        torch.cuda.synchronize()
        img = bf.r.image(0).cpu().numpy()
        bf.close()
        worst, frac = assert_image_parity(img, ref)
        print(f"C2 (tile {tile}, bins {bins}): worst {worst:.2e}, flagged {frac:.2e}")


@pytest.mark.slow
def test_render_c3_full_frame():
    """The 6M-Gaussian 4K frame (the large-scene workload): pair count against the oracle's and every one of
    its 8.3 M pixels against the oracle's image (the oracle's loops over tiles run on the host's cores)."""
    import torch
    from paper_2602_03207_amd import binding as B
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    scene, cam = scenegen.c3()
    g = GaussianTensors.from_scene(scene)
    r = Renderer([cam], gpu_options(sh_degree=3, flags=B.WS_FLAG_DEPTH_FIRST))
    r.forward(g)
    torch.cuda.synchronize()
    assert r.status() == 0
    img = r.image(0).cpu().numpy()
    ro = oracle_options(sh_degree=3)
    m_ref = oracle.pair_count(scene, cam, ro)
    assert abs(r.num_pairs - m_ref) <= 1e-4 * m_ref, (r.num_pairs, m_ref)  # rectangle bounds at a margin
    print("C3: oracle render of the full frame", flush=True)
    ref = oracle.render(scene, cam, ro, outcomes=True)
    worst, frac = assert_image_parity(img, ref)
    del ref
    # the fastest 4K layout (16x16 tiles in 4x2 bins, 32-bit keys, device-sized sequence): the same image
    m_gpu = r.num_pairs
    del r
    rb = Renderer([cam], gpu_options(sh_degree=3, flags=B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32, bin_x=4,
                                     bin_y=2))
    m = rb.forward(g)
    rb._ensure_capacity(int(m * 1.1) + 4096)
    rb.forward_capacity(g)
    torch.cuda.synchronize()
    assert rb.status() == 0
    assert np.array_equal(rb.image(0).cpu().numpy().view(np.uint32), img.view(np.uint32))
    print(f"C3: worst {worst:.2e}, several outcomes on {frac:.2e} of pixels, M gpu {m_gpu} oracle {m_ref}")


@pytest.mark.slow
def test_render_c4_all_views_one_launch():
    """The 64-view workload of uneven resolution rendered as one batched call in the layouts the multi-view
    benchmark's autotuner picks among (here 16x16 tiles in 4x2 bins with 32-bit keys and one workgroup per
    tile, and 32x16 tiles with the persistent ordered render): one view of each size, every pixel against the
    oracle's image of that view; both layouts give identical images of all 64 views."""
    import torch
    from paper_2602_03207_amd import binding as B
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    scene, cams = scenegen.c4()
    g = GaussianTensors.from_scene(scene)
    r = Renderer(cams, gpu_options(sh_degree=3, tile_w=16, tile_h=16, radix_bits=8, bin_x=4, bin_y=2,
                                   flags=B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32))
    m = r.forward(g)
    r._ensure_capacity(int(m * 1.1) + 4096)
    r.forward_capacity(g)
    torch.cuda.synchronize()
    assert r.status() == 0
    sizes = {}
    for v, c in enumerate(cams):
        sizes.setdefault((c.width, c.height), v)
    ro = oracle_options(sh_degree=3)
    for v in sorted(sizes.values()):
        cam = cams[v]
        img = r.image(v).cpu().numpy()
        ref = oracle.render(scene, cam, ro, outcomes=True)
        worst, frac = assert_image_parity(img, ref)
        print(f"C4 view {v} ({cam.width}x{cam.height}): worst {worst:.2e}, flagged {frac:.2e}")
    images = r.images.clone()
    del r
    ro_r = Renderer(cams, gpu_options(sh_degree=3, tile_w=32, tile_h=16, radix_bits=6,
                                      flags=B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_ORDERED_RENDER))
    ro_r.forward(g)
    torch.cuda.synchronize()
    assert ro_r.status() == 0
    assert torch.equal(ro_r.images.view(torch.int32), images.view(torch.int32))


def test_invariance_tile_size_radix_width_and_emission_order():
    from paper_2602_03207_amd import binding as B
    scene, cam = scenegen.c1()
    base = _full(scene, [cam]).image(0).cpu().numpy()
    for tile in ((8, 8), (16, 8), (16, 16), (32, 16)):
        for rb in (4, 8):
            for flags in (0, B.WS_FLAG_DEPTH_FIRST):
                img = _full(scene, [cam], tile_w=tile[0], tile_h=tile[1], radix_bits=rb,
                            flags=flags).image(0).cpu().numpy()
                assert np.array_equal(img.view(np.uint32), base.view(np.uint32)), (tile, rb, flags)


def test_invariance_repeat_and_permutation():
    scene, cam = scenegen.c1()
    a = _full(scene, [cam]).image(0).cpu().numpy()
    b = _full(scene, [cam]).image(0).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    # keep the Gaussians whose fp32 depth is unique, so that the order cannot depend on ids
    ref = oracle.preprocess(scene, cam, oracle_options())
    _, first, counts = np.unique(ref["depth32"], return_index=True, return_counts=True)
    keep = np.sort(first[counts == 1])
    base = scene.subset(keep)
    a = _full(base, [cam]).image(0).cpu().numpy()
    perm = np.random.default_rng(0).permutation(base.n)
    c = _full(base.subset(perm), [cam]).image(0).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), c.view(np.uint32))


def test_batched_views_equal_single_views():
    scene, _ = scenegen.c1()
    cams = [scenegen.look_at([0, 0, -3], [0, 0, 0], 128, 96), scenegen.look_at([1.5, -0.5, -2.5], [0, 0, 0], 70, 130),
            scenegen.look_at([-2.5, 0.3, -1.5], [0, 0, 0], 256, 64)]
    rb = _full(scene, cams)
    for v, cam in enumerate(cams):
        single = _full(scene, [cam]).image(0).cpu().numpy()
        assert np.array_equal(rb.image(v).cpu().numpy().view(np.uint32), single.view(np.uint32)), v


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 16)])
def test_ordered_persistent_render_equals_plain(tile):
    """WS_FLAG_ORDERED_RENDER (persistent workgroups, longest tiles first) changes no pixel."""
    from paper_2602_03207_amd import binding as B
    scene, _ = scenegen.c1()
    cams = [scenegen.look_at([0, 0, -3], [0, 0, 0], 256, 256), scenegen.look_at([1.5, -0.5, -2.5], [0, 0, 0], 70, 130),
            scenegen.look_at([-0.4, 0.3, -1.2], [0, 0, 0], 333, 97)]
    kw = dict(tile_w=tile[0], tile_h=tile[1])
    plain = _full(scene, cams, **kw)
    ordered = _full(scene, cams, flags=B.WS_FLAG_ORDERED_RENDER, **kw)
    assert ordered.status() == 0
    assert np.array_equal(ordered.images.cpu().numpy().view(np.uint32), plain.images.cpu().numpy().view(np.uint32))
    # and against the oracle on the first view
    ref = oracle.render(scene, cams[0], oracle_options(*tile), outcomes=True)
    assert_image_parity(ordered.image(0).cpu().numpy(), ref)


@pytest.mark.parametrize("flags", [1, 2, 3])
def test_ablation_flags_match_oracle(flags):
    """Fixed 3-sigma extent (1) and no viewport cull (2), the ablations of Sec. 4.4, against the oracle."""
    scene = scenegen.random_scene(4000, 31, mean_lo=-1.5, mean_hi=1.5, log_scale_mu=-3.0, log_scale_sd=0.6,
                                  logit_sd=2.5, sh_degree=1, dc_sd=0.5, rest_sd=0.2)
    cam = scenegen.look_at([0.3, 0.2, -1.4], [0, 0, 0.5], 150, 110)
    r = _full(scene, [cam], flags=flags)
    ref = oracle.render(scene, cam, oracle_options(sh_degree=1, flags=flags), outcomes=True)
    assert r.num_pairs == ref["keys"].size
    assert_image_parity(r.image(0).cpu().numpy(), ref)
