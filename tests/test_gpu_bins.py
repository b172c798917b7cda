"""Bins of tiles as the key cells: ws_preprocess keys name bins, ws_sort orders the bin bits and
ws_expand_bins rebuilds every tile's list from its bin's list (Sec. 3.2: a tile lists the splats whose
footprint meets it, in depth order).

The pins: the bin pairs equal the oracle's pairs for cells of the bin's pixel size (the oracle's emission
rule at another cell size); where the key carries the mask of the bin's tiles that a splat covers, that
mask equals the tiles the oracle lists the splat in; every expanded tile list equals, id for id, that
tile's run of pairs in the path whose keys name tiles (the oracle's tile-sorted pairs for a single view),
and images are identical to the bit."""
import math

import numpy as np
import pytest

import oracle
import scenegen
from _helpers import gpu_options, oracle_options

pytestmark = pytest.mark.gpu


def _renderer(scene, cams, **kw):
    import torch
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    r = Renderer(cams, gpu_options(sh_degree=scene.sh_degree, **kw))
    r.forward(GaussianTensors.from_scene(scene))
    torch.cuda.synchronize()
    assert r.status() == 0
    return r


def _lists(r):
    """Per-tile id lists of a renderer (the tile's run of pairs, or its expanded list)."""
    rng = r.tile_ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    vals = r.lists.cpu().numpy().view(np.uint32)
    return [vals[a:b] for a, b in rng]


def _multiview():
    scene = scenegen.random_scene(6000, 12, log_scale_mu=-3.0, sh_degree=1, dc_sd=0.4, rest_sd=0.2)
    cams = [scenegen.look_at([0, 0, -3], [0, 0, 0], 100, 80), scenegen.look_at([2, -1, -2], [0, 0, 0], 64, 120),
            scenegen.look_at([-1, 2, -3], [0, 0, 0], 200, 150)]
    return scene, cams


def _mask_shift(total_bins, per_bin):
    """Where the bins' coverage mask starts in a key's cell word: above the bin id's bits, if both fit in
    32 bits (-1: the keys carry no mask)."""
    bits = max(1, math.ceil(math.log2(max(total_bins, 2))))
    return bits if bits + per_bin <= 32 else -1


def _split_words(words, shift):
    words = words.astype(np.uint64)
    if shift < 0:
        return words, None
    return words & np.uint64((1 << shift) - 1), words >> np.uint64(shift)


def _expected_masks(scene, cam, tile, bins):
    """(Gaussian id, bin) -> mask of the bin's tiles (bit row * bin_x + col) in the oracle's tile-level pairs."""
    ro = oracle_options(tile_w=tile[0], tile_h=tile[1])
    kt, vt = oracle.emit(scene, cam, ro)
    ntx, _ = oracle.tiles_xy(cam, ro)
    t = (kt >> np.uint64(32)).astype(np.int64)
    tx, ty = t % ntx, t // ntx
    bx, by = tx // bins[0], ty // bins[1]
    nbx = -(-ntx // bins[0])
    bid = by * nbx + bx
    bit = (ty - by * bins[1]) * bins[0] + (tx - bx * bins[0])
    out = {}
    for gid, b, bt in zip(vt.tolist(), bid.tolist(), bit.tolist()):
        out[(gid, b)] = out.get((gid, b), 0) | (1 << bt)
    return out


@pytest.mark.parametrize("mode", ["gaussian_order", "depth_first", "keys32"])
@pytest.mark.parametrize("tile,bins", [((16, 16), (2, 2)), ((32, 16), (4, 4)), ((8, 8), (8, 4)), ((16, 8), (1, 8))])
def test_bin_pairs_match_the_oracle_at_the_bin_size(tile, bins, mode):
    from paper_2602_03207_amd import binding as B
    scene, cam = scenegen.c1()
    flags = {"gaussian_order": 0, "depth_first": B.WS_FLAG_DEPTH_FIRST,
             "keys32": B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32}[mode]
    r = _renderer(scene, [cam], tile_w=tile[0], tile_h=tile[1], bin_x=bins[0], bin_y=bins[1], flags=flags)
    cell = oracle_options(tile_w=tile[0] * bins[0], tile_h=tile[1] * bins[1])
    keys, vals = oracle.emit(scene, cam, cell)
    m = r.num_pairs
    assert m == keys.size
    tt = r.tiles_touched.cpu().numpy().astype(np.int64)
    assert tt.sum() == m
    shift = _mask_shift(r.total_bins, bins[0] * bins[1])
    assert (shift >= 0) == (bins[0] * bins[1] <= 16)  # every bin size here but 8 x 4 carries the mask

    def cells_and_masks(t):
        a = t[:m].cpu().numpy()
        if mode == "keys32":
            return _split_words(a.view(np.uint32), shift), None
        k = a.view(np.uint64)
        return _split_words((k >> np.uint64(32)).astype(np.uint32), shift), k & np.uint64(0xFFFFFFFF)

    sk, sv = oracle.stable_sort(keys, vals)
    (cells, masks), depth = cells_and_masks(r.keys_b)
    gv = r.vals_b[:m].cpu().numpy().view(np.uint32)
    assert np.array_equal(gv, sv)
    assert np.array_equal(cells, sk >> np.uint64(32))
    if depth is not None:
        assert np.array_equal(depth, sk & np.uint64(0xFFFFFFFF))
    if masks is not None:
        # every pair's mask holds exactly the bin's tiles that the oracle lists the splat in
        want = _expected_masks(scene, cam, tile, bins)
        assert len(want) == m
        got = {(int(v), int(c)): int(mk) for v, c, mk in zip(gv, cells, masks)}
        assert got == want
    if mode == "gaussian_order":
        (cells_a, _), depth_a = cells_and_masks(r.keys_a)
        assert np.array_equal((cells_a << np.uint64(32)) | depth_a, keys)
        assert np.array_equal(r.vals_a[:m].cpu().numpy().view(np.uint32), vals)


@pytest.mark.parametrize("tile,bins", [((16, 16), (2, 2)), ((32, 16), (4, 4)), ((8, 8), (4, 8)), ((16, 8), (8, 1))])
def test_expanded_lists_equal_the_oracle_tile_lists(tile, bins):
    """Single view: each tile's expanded list is the oracle's tile-sorted run of that tile."""
    from paper_2602_03207_amd import binding as B
    scene, cam = scenegen.c1()
    r = _renderer(scene, [cam], tile_w=tile[0], tile_h=tile[1], bin_x=bins[0], bin_y=bins[1],
                  flags=B.WS_FLAG_DEPTH_FIRST)
    ro = oracle_options(tile_w=tile[0], tile_h=tile[1])
    keys, vals = oracle.emit(scene, cam, ro)
    sk, sv = oracle.stable_sort(keys, vals)
    tx, ty = oracle.tiles_xy(cam, ro)
    ref = oracle.tile_ranges(sk, tx * ty)
    got = _lists(r)
    assert len(got) == tx * ty
    for t in range(tx * ty):
        want = sv[ref[t, 0]:ref[t, 1]]
        assert np.array_equal(got[t], want), t
    # the slots of one bin never overlap another bin's
    rng = r.tile_ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    assert (rng[:, 1] >= rng[:, 0]).all() and rng[:, 1].max() <= r.per_bin * r.capacity


@pytest.mark.parametrize("depth_first", [False, True])
@pytest.mark.parametrize("tile,bins", [((16, 16), (4, 4)), ((32, 16), (2, 4)), ((8, 8), (8, 8))])
def test_binned_multiview_lists_and_images_equal_tile_keys(tile, bins, depth_first):
    """Three views of uneven size (partial bins on every right / bottom edge): lists and images of the
    binned path equal those of the path whose keys name tiles."""
    import torch
    from paper_2602_03207_amd import binding as B
    scene, cams = _multiview()
    flags = B.WS_FLAG_DEPTH_FIRST if depth_first else 0
    a = _renderer(scene, cams, tile_w=tile[0], tile_h=tile[1], flags=flags)
    b = _renderer(scene, cams, tile_w=tile[0], tile_h=tile[1], bin_x=bins[0], bin_y=bins[1], flags=flags)
    assert b.total_bins < a.total_tiles and b.num_pairs < a.num_pairs
    la, lb = _lists(a), _lists(b)
    assert len(la) == len(lb) == a.total_tiles
    for t in range(a.total_tiles):
        assert np.array_equal(la[t], lb[t]), t
    assert torch.equal(a.images.view(torch.int32), b.images.view(torch.int32))


def test_binned_ordered_render_and_graph_replay_equal_plain():
    import torch
    from paper_2602_03207_amd import binding as B
    from paper_2602_03207_amd.batched import BatchedForward
    from paper_2602_03207_amd.pipeline import GaussianTensors
    scene, cams = _multiview()
    base = _renderer(scene, cams, tile_w=16, tile_h=16)
    k32 = B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32
    for flags in (B.WS_FLAG_DEPTH_FIRST, B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_ORDERED_RENDER, k32,
                  k32 | B.WS_FLAG_ORDERED_RENDER):
        opts = gpu_options(sh_degree=scene.sh_degree, tile_w=16, tile_h=16, bin_x=4, bin_y=2, flags=flags)
        bf = BatchedForward(cams, opts, GaussianTensors.from_scene(scene))
        for _ in range(3):
            bf.replay()
            bf.check()
            assert torch.equal(bf.r.images.view(torch.int32), base.images.view(torch.int32))
        bf.close()


def test_binned_backward_equals_tile_keys():
    """The backward reads the expanded lists: its gradients equal those of the path whose keys name
    tiles, up to the order of the floating-point atomics."""
    import torch
    from paper_2602_03207_amd.pipeline import GaussianTensors
    scene, cams = _multiview()
    g = GaussianTensors.from_scene(scene)
    a = _renderer(scene, cams, tile_w=16, tile_h=16)
    b = _renderer(scene, cams, tile_w=16, tile_h=16, bin_x=2, bin_y=4)
    dL = torch.randn(a.images.numel(), generator=torch.Generator().manual_seed(5)).to(a.images.device)
    ga = a.backward(g, dL)
    gb = b.backward(g, dL)
    torch.cuda.synchronize()
    for k in ga:
        x, y = ga[k].double(), gb[k].double()
        err = ((x - y).abs().max() / max(x.abs().max().item(), 1e-30)).item()
        assert err < 1e-5, (k, err)


def test_binned_empty_scene_and_capacity_overflow():
    import torch
    from paper_2602_03207_amd import binding as B
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    scene, cams = _multiview()
    # every splat behind the cameras: no pairs, every tile list empty, background everywhere
    far = scenegen.random_scene(500, 3, sh_degree=1)
    far.means[2] = -50.0
    r = _renderer(far, cams, tile_w=16, tile_h=16, bin_x=4, bin_y=4, bg=(0.25, 0.5, 0.75))
    assert r.num_pairs == 0
    rng = r.tile_ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    assert (rng[:, 0] == rng[:, 1]).all()
    for v in range(len(cams)):
        img = r.image(v).cpu().numpy()
        assert np.array_equal(img, np.broadcast_to(np.array([0.25, 0.5, 0.75], np.float32)[:, None, None], img.shape))
    # a capacity below M: the device status reports it and the expansion writes nothing
    opts = gpu_options(sh_degree=scene.sh_degree, tile_w=16, tile_h=16, bin_x=2, bin_y=2)
    rr = Renderer(cams, opts, capacity=1024)
    g = GaussianTensors.from_scene(scene)
    rr.tile_ranges.fill_(7)
    rr.d_status.zero_()
    rr.preprocess(g)
    m = int(rr.d_num_pairs.item())
    assert m > 1024
    rr.sort(rr.capacity, device_count=True)
    rr.render(rr.capacity)
    torch.cuda.synchronize()
    assert rr.status() == B.WS_ERR_CAPACITY
    assert (rr.tile_ranges.cpu().numpy() == 7).all()
