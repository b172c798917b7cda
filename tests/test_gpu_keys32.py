"""32-bit keys (WS_FLAG_KEYS32) and ws_sort32.

With depth-first emission the pairs already come in depth order, so a key only has to name the tile:
ws_preprocess writes the tile id alone and ws_sort32 orders those 32 bits.  The pins: ws_sort32 is
bit-exact against the oracle's std::stable_sort on the same keys (widened to 64 bits, same bit range);
the 32-bit keys equal the high words of the oracle's pairs, and after the sort the ids equal the oracle's
stable-sorted pairs; ranges, lists and images are identical to the bit to those of 64-bit keys, for every
tile size and radix width, on the plain and the device-sized sequences, and with bins of tiles."""
import numpy as np
import pytest

import oracle
import scenegen
from _helpers import gpu_options, oracle_options

pytestmark = pytest.mark.gpu


def _gpu_sort32(keys, vals, begin_bit, end_bit, radix_bits=0, capacity=None, device_count=False):
    import torch
    from paper_2602_03207_amd import binding as B
    n = keys.size
    cap = capacity if capacity is not None else n
    print(f"ws_sort32 n={n} bits=[{begin_bit},{end_bit}) radix={radix_bits} cap={cap}", flush=True)
    kin = torch.zeros(max(cap, 1), dtype=torch.int32, device="cuda")
    vin = torch.zeros(max(cap, 1), dtype=torch.int32, device="cuda")
    kin[:n] = torch.from_numpy(keys.view(np.int32))
    vin[:n] = torch.from_numpy(vals.view(np.int32))
    kout = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
    vout = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
    d_n = torch.tensor([n], dtype=torch.int64, device="cuda")
    d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
    need = B.ws_sort32_workspace_size(max(cap, 1), begin_bit, end_bit, radix_bits)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    B.ws_sort32(kin, vin, kout, vout, cap if device_count else n, d_n if device_count else None, d_status,
                begin_bit, end_bit, radix_bits, ws, ws.numel())
    torch.cuda.synchronize()
    assert int(d_status.item()) == 0
    return kout[:n].cpu().numpy().view(np.uint32), vout[:n].cpu().numpy().view(np.uint32)


def _oracle_sort32(keys, vals, b0, b1):
    k, v = oracle.stable_sort(keys.astype(np.uint64), vals, b0, b1)
    return k.astype(np.uint32), v


def _cases():
    rng = np.random.default_rng(32)
    yield "n1", rng.integers(0, 2**32, 1, dtype=np.uint64).astype(np.uint32)
    for n in (63, 64, 65, 1023, 1024, 1025, 4095, 4096, 4097, 100_003):
        yield f"rand{n}", rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    yield "equal", np.full(20_000, 7, np.uint32)
    yield "sorted", (np.arange(30_000, dtype=np.uint64) * np.uint64(977)).astype(np.uint32)
    yield "reversed", (np.arange(30_000, dtype=np.uint64) * np.uint64(977)).astype(np.uint32)[::-1].copy()
    yield "bit0", rng.integers(0, 2, 50_000, dtype=np.uint64).astype(np.uint32)
    yield "top", (rng.integers(0, 2, 50_000, dtype=np.uint64) << np.uint64(31)).astype(np.uint32)
    yield "tiles", rng.integers(0, 8160, 70_000, dtype=np.uint64).astype(np.uint32)


@pytest.mark.parametrize("bits", [(0, 32), (0, 13), (5, 19), (31, 32)])
def test_sort32_bit_exact(bits):
    b0, b1 = bits
    for name, keys in _cases():
        vals = np.arange(keys.size, dtype=np.uint32)
        want_k, want_v = _oracle_sort32(keys, vals, b0, b1)
        got_k, got_v = _gpu_sort32(keys, vals, b0, b1)
        assert np.array_equal(got_v, want_v), (name, bits)
        assert np.array_equal(got_k, want_k), (name, bits)


@pytest.mark.parametrize("radix_bits", [1, 3, 4, 5, 6, 7, 8, 9, 10])
def test_sort32_every_radix_width(radix_bits):
    rng = np.random.default_rng(100 + radix_bits)
    keys = rng.integers(0, 2**32, 60_001, dtype=np.uint64).astype(np.uint32)
    vals = rng.integers(0, 2**32, keys.size, dtype=np.uint64).astype(np.uint32)
    want_k, want_v = _oracle_sort32(keys, vals, 0, 32)
    got_k, got_v = _gpu_sort32(keys, vals, 0, 32, radix_bits)
    assert np.array_equal(got_k, want_k) and np.array_equal(got_v, want_v)


def test_sort32_large_schedule_and_device_count():
    # capacities above 2^20 take the wait-free schedule (per-pass digit tables), smaller ones the look-back
    rng = np.random.default_rng(7)
    keys = rng.integers(0, 1 << 15, 1_500_001, dtype=np.uint64).astype(np.uint32)
    vals = np.arange(keys.size, dtype=np.uint32)
    want_k, want_v = _oracle_sort32(keys, vals, 0, 15)
    for cap, dc, rb in ((keys.size, False, 8), (2_000_000, True, 8), (keys.size, False, 10), (2_000_000, True, 9)):
        got_k, got_v = _gpu_sort32(keys, vals, 0, 15, radix_bits=rb, capacity=cap, device_count=dc)
        assert np.array_equal(got_k, want_k) and np.array_equal(got_v, want_v)
    # the frame's case: 9-10 bits of bin ids sorted in one pass of the look-back schedule
    bins = rng.integers(0, 1 << 10, 700_001, dtype=np.uint64).astype(np.uint32)
    want_k, want_v = _oracle_sort32(bins, vals[:bins.size], 0, 10)
    got_k, got_v = _gpu_sort32(bins, vals[:bins.size], 0, 10, radix_bits=10, capacity=900_000, device_count=True)
    assert np.array_equal(got_k, want_k) and np.array_equal(got_v, want_v)
    small = keys[:123_457].copy()
    want_k, want_v = _oracle_sort32(small, vals[:small.size], 0, 15)
    outs = [_gpu_sort32(small, vals[:small.size], 0, 15, capacity=300_000, device_count=True) for _ in range(3)]
    for got_k, got_v in outs:
        assert np.array_equal(got_k, want_k) and np.array_equal(got_v, want_v)


def _frame(scene, cams, capacity_path=False, **kw):
    import torch
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    print(f"frame {kw} capacity_path={capacity_path}", flush=True)
    r = Renderer(cams, gpu_options(sh_degree=scene.sh_degree, **kw))
    g = GaussianTensors.from_scene(scene)
    m = r.forward(g)
    if capacity_path:
        r._ensure_capacity(int(m * 1.1) + 4096)
        r.forward_capacity(g)
    torch.cuda.synchronize()
    assert r.status() == 0
    return r


def test_keys32_are_the_tile_words_of_the_oracle_pairs():
    from paper_2602_03207_amd import binding as B
    scene, cam = scenegen.c1()
    r = _frame(scene, [cam], flags=B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32)
    keys, vals = oracle.emit(scene, cam, oracle_options())
    m = r.num_pairs
    assert m == keys.size and r.keys_a.dtype.itemsize == 4
    # emission in (depth, entry) order: the ids and tiles of the oracle's pairs regrouped that way
    from test_gpu_preprocess import _depth_first_reference
    wk, wv = _depth_first_reference(keys, vals)
    assert np.array_equal(r.vals_a[:m].cpu().numpy().view(np.uint32), wv)
    assert np.array_equal(r.keys_a[:m].cpu().numpy().view(np.uint32), (wk >> np.uint64(32)).astype(np.uint32))
    # the sort of the tile bits gives the oracle's stable (tile, depth) order
    sk, sv = oracle.stable_sort(keys, vals)
    assert np.array_equal(r.vals_b[:m].cpu().numpy().view(np.uint32), sv)
    assert np.array_equal(r.keys_b[:m].cpu().numpy().view(np.uint32), (sk >> np.uint64(32)).astype(np.uint32))
    n_tiles = int(np.prod(oracle.tiles_xy(cam, oracle_options())))
    want_ranges = oracle.tile_ranges(sk, n_tiles)
    got = r.tile_ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    assert np.array_equal(got.astype(np.int64), np.asarray(want_ranges, np.int64).reshape(-1, 2))


@pytest.mark.parametrize("tile,radix", [((16, 16), 8), ((32, 16), 6), ((8, 8), 5), ((16, 8), 7)])
@pytest.mark.parametrize("capacity_path", [False, True])
def test_keys32_frame_identical_to_64bit_keys(tile, radix, capacity_path):
    from paper_2602_03207_amd import binding as B
    scene = scenegen.random_scene(8000, 21, log_scale_mu=-3.1, sh_degree=2, dc_sd=0.4, rest_sd=0.2)
    cams = [scenegen.look_at([0, 0, -3], [0, 0, 0], 300, 200), scenegen.look_at([2, -1, -2], [0, 0, 0], 130, 250),
            scenegen.look_at([-1, 2, -3], [0, 0, 0], 77, 61)]
    kw = dict(tile_w=tile[0], tile_h=tile[1], radix_bits=radix)
    a = _frame(scene, cams, capacity_path, flags=B.WS_FLAG_DEPTH_FIRST, **kw)
    b = _frame(scene, cams, capacity_path, flags=B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32, **kw)
    m = a.num_pairs
    assert b.num_pairs == m and m > 0
    ka = a.keys_b[:m].cpu().numpy().view(np.uint64)
    assert np.array_equal(b.keys_b[:m].cpu().numpy().view(np.uint32), (ka >> np.uint64(32)).astype(np.uint32))
    assert np.array_equal(a.vals_b[:m].cpu().numpy(), b.vals_b[:m].cpu().numpy())
    assert np.array_equal(a.tile_ranges.cpu().numpy(), b.tile_ranges.cpu().numpy())
    assert np.array_equal(a.images.cpu().numpy().view(np.uint32), b.images.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("tile,bins", [((16, 16), (2, 2)), ((32, 16), (4, 4))])
def test_keys32_with_bins(tile, bins):
    from paper_2602_03207_amd import binding as B
    scene = scenegen.random_scene(6000, 12, log_scale_mu=-3.0, sh_degree=1, dc_sd=0.4, rest_sd=0.2)
    cams = [scenegen.look_at([0, 0, -3], [0, 0, 0], 100, 80), scenegen.look_at([2, -1, -2], [0, 0, 0], 64, 120)]
    kw = dict(tile_w=tile[0], tile_h=tile[1])
    plain = _frame(scene, cams, flags=B.WS_FLAG_DEPTH_FIRST, **kw)
    binned = _frame(scene, cams, flags=B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32, bin_x=bins[0], bin_y=bins[1], **kw)
    rp = plain.tile_ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    rb = binned.tile_ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    vp = plain.lists.cpu().numpy().view(np.uint32)
    vb = binned.lists.cpu().numpy().view(np.uint32)
    for (a0, a1), (b0, b1) in zip(rp, rb):
        assert np.array_equal(vp[a0:a1], vb[b0:b1])
    assert np.array_equal(plain.images.cpu().numpy().view(np.uint32), binned.images.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("n", [5000, 1_500_000])  # look-back and wait-free schedules
def test_sort32_respects_status_word(n):
    import torch
    from paper_2602_03207_amd import binding as B
    kin = torch.arange(n, 0, -1, dtype=torch.int32, device="cuda")
    vin = torch.arange(n, dtype=torch.int32, device="cuda")
    kout = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    vout = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    d_status = torch.tensor([B.WS_ERR_CAPACITY], dtype=torch.int32, device="cuda")
    need = B.ws_sort32_workspace_size(n, 0, 32, 0)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    print(f"ws_sort32 with a set status word, n={n}", flush=True)
    B.ws_sort32(kin, vin, kout, vout, n, None, d_status, 0, 32, 0, ws, ws.numel())
    torch.cuda.synchronize()
    assert bool((kout == -1).all()) and bool((vout == -1).all())
    assert int(d_status.item()) == B.WS_ERR_CAPACITY


@pytest.mark.parametrize("bins", [(1, 1), (4, 2)])
def test_keys32_empty_frame_and_capacity_overflow(bins):
    """32-bit keys at the edges: a frame without pairs renders the background with every range empty; a
    capacity below M is reported in the status word on the device-sized path and nothing downstream writes."""
    import torch
    from paper_2602_03207_amd import binding as B
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    flags = B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32
    cams = [scenegen.look_at([0, 0, -3], [0, 0, 0], 100, 80), scenegen.look_at([2, -1, -2], [0, 0, 0], 64, 120)]
    far = scenegen.random_scene(500, 3, sh_degree=1)
    far.means[2] = -50.0  # behind both cameras
    print(f"keys32 empty frame, bins {bins}", flush=True)
    r = _frame(far, cams, bin_x=bins[0], bin_y=bins[1], flags=flags, bg=(0.25, 0.5, 0.75))
    assert r.num_pairs == 0
    rng_ = r.tile_ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    assert (rng_[:, 0] == rng_[:, 1]).all()
    for v in range(len(cams)):
        img = r.image(v).cpu().numpy()
        assert np.array_equal(img, np.broadcast_to(np.array([0.25, 0.5, 0.75], np.float32)[:, None, None], img.shape))
    scene = scenegen.random_scene(6000, 12, log_scale_mu=-3.0, sh_degree=1, dc_sd=0.4, rest_sd=0.2)
    print(f"keys32 capacity overflow, bins {bins}", flush=True)
    rr = Renderer(cams, gpu_options(sh_degree=1, bin_x=bins[0], bin_y=bins[1], flags=flags), capacity=1024)
    g = GaussianTensors.from_scene(scene)
    rr.tile_ranges.fill_(7)
    rr.images.fill_(-1.0)
    rr.d_status.zero_()
    rr.preprocess(g)
    assert int(rr.d_num_pairs.item()) > 1024
    rr.sort(rr.capacity, device_count=True)
    rr.render(rr.capacity)
    torch.cuda.synchronize()
    assert rr.status() == B.WS_ERR_CAPACITY
    assert (rr.tile_ranges.cpu().numpy() == 7).all() and bool((rr.images == -1.0).all())
    # the plain sequence grows its buffers and renders the same image as 64-bit keys
    m = rr.forward(g)
    torch.cuda.synchronize()
    assert rr.status() == 0 and m > 1024
    ref = _frame(scene, cams, bin_x=bins[0], bin_y=bins[1], flags=B.WS_FLAG_DEPTH_FIRST)
    assert torch.equal(rr.images.view(torch.int32), ref.images.view(torch.int32))


def test_keys32_single_pair():
    """One visible splat covering one tile: one pair, one non-empty range, the oracle's pixels."""
    from paper_2602_03207_amd import binding as B
    scene = scenegen.random_scene(1, 5, sh_degree=0, log_scale_mu=-5.0, log_scale_sd=0.0)
    scene.means[:, 0] = [0.1, 0.1, 0.0]  # centre at pixel (33.8, 33.8): its rectangle stays inside one tile
    scene.opacity_logits[0] = 4.0
    cam = scenegen.look_at([0, 0, -3], [0, 0, 0], 64, 64)
    r = _frame(scene, [cam], flags=B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32)
    keys, vals = oracle.emit(scene, cam, oracle_options())
    assert r.num_pairs == keys.size == 1
    assert np.array_equal(r.keys_b[:r.num_pairs].cpu().numpy().view(np.uint32),
                          (np.sort(keys) >> np.uint64(32)).astype(np.uint32))
    ref = oracle.render(scene, cam, oracle_options())
    err = np.abs(r.image(0).cpu().numpy().astype(np.float64) - ref["rgb"]).max()
    assert err < 2e-4, err
