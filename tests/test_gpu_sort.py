"""ws_sort on the GPU: bit-exact against the oracle's std::stable_sort, identical run to run."""
import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu


def _gpu_sort(keys, vals, begin_bit, end_bit, radix_bits=0, capacity=None, device_count=False):
    import torch
    from paper_2602_03207_amd import binding as B
    n = keys.size
    cap = capacity if capacity is not None else n
    kin = torch.zeros(max(cap, 1), dtype=torch.int64, device="cuda")
    vin = torch.zeros(max(cap, 1), dtype=torch.int32, device="cuda")
    kin[:n] = torch.from_numpy(keys.view(np.int64))
    vin[:n] = torch.from_numpy(vals.view(np.int32))
    kout = torch.full((max(cap, 1),), -1, dtype=torch.int64, device="cuda")
    vout = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
    d_n = torch.tensor([n], dtype=torch.int64, device="cuda")
    d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
    need = B.ws_sort_workspace_size(max(cap, 1), begin_bit, end_bit, radix_bits)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    B.ws_sort(kin, vin, kout, vout, cap if device_count else n, d_n if device_count else None, d_status, begin_bit,
              end_bit, radix_bits, ws, ws.numel())
    torch.cuda.synchronize()
    assert int(d_status.item()) == 0
    return kout[:n].cpu().numpy().view(np.uint64), vout[:n].cpu().numpy().view(np.uint32)


def _cases():
    rng = np.random.default_rng(5)
    yield "n1", rng.integers(0, 2**63, 1, dtype=np.uint64)
    for n in (63, 64, 65, 4095, 4096, 4097, 100_003):
        yield f"rand{n}", rng.integers(0, 2**63, n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n, dtype=np.uint64)
    yield "equal", np.full(20_000, 7, np.uint64)
    yield "sorted", np.arange(30_000, dtype=np.uint64) * np.uint64(977)
    yield "reversed", (np.arange(30_000, dtype=np.uint64) * np.uint64(977))[::-1].copy()
    yield "high32", rng.integers(0, 300, 50_000, dtype=np.uint64) << np.uint64(32)
    yield "bit0", rng.integers(0, 2, 50_000, dtype=np.uint64)
    yield "tiledepth", (rng.integers(0, 8160, 70_000, dtype=np.uint64) << np.uint64(32)) | \
        rng.integers(0x3F000000, 0x41000000, 70_000, dtype=np.uint64)


@pytest.mark.parametrize("bits", [(0, 64), (0, 45), (3, 17), (32, 64), (63, 64)])
def test_sort_adversarial_bit_exact(bits):
    b0, b1 = bits
    for name, keys in _cases():
        vals = np.arange(keys.size, dtype=np.uint32)
        want_k, want_v = oracle.stable_sort(keys, vals, b0, b1)
        got_k, got_v = _gpu_sort(keys, vals, b0, b1)
        assert np.array_equal(got_v, want_v), (name, bits)
        assert np.array_equal(got_k, want_k), (name, bits)


@pytest.mark.parametrize("radix_bits", [1, 3, 4, 5, 6, 7, 8])
def test_sort_every_radix_width(radix_bits):
    rng = np.random.default_rng(radix_bits)
    keys = (rng.integers(0, 5000, 60_001, dtype=np.uint64) << np.uint64(32)) | rng.integers(0, 2**31, 60_001, dtype=np.uint64)
    vals = rng.integers(0, 2**32, keys.size, dtype=np.uint64).astype(np.uint32)
    want_k, want_v = oracle.stable_sort(keys, vals, 0, 45)
    got_k, got_v = _gpu_sort(keys, vals, 0, 45, radix_bits)
    assert np.array_equal(got_k, want_k) and np.array_equal(got_v, want_v)


@pytest.mark.parametrize("bits,radix_bits,n,capacity", [
    ((0, 20), 10, 200_003, None),        # look-back schedule, two 10-bit passes
    ((5, 32), 9, 150_001, None),         # look-back, three 9-bit passes
    ((0, 32), 10, 150_001, None),        # look-back: 10 bits narrowed until the histograms fit
    ((0, 30), 10, 1_500_001, None),      # wait-free schedule, three 10-bit passes
    ((32, 51), 10, 1_200_001, 1_600_000),  # wait-free, device-sized, a 10-bit and a 9-bit pass
])
def test_sort_wide_digits(bits, radix_bits, n, capacity):
    """Digits wider than the 256 threads of a sort tile (9 and 10 bits: several digits per thread in the
    per-digit scans and look-backs) on both schedules, bit-exact against std::stable_sort."""
    rng = np.random.default_rng(radix_bits * 1000 + bits[0])
    keys = rng.integers(0, 2**63, n, dtype=np.uint64)
    keys[::7] = keys[3]  # runs of equal keys: stability
    vals = np.arange(n, dtype=np.uint32)
    want_k, want_v = oracle.stable_sort(keys, vals, *bits)
    got_k, got_v = _gpu_sort(keys, vals, *bits, radix_bits=radix_bits, capacity=capacity,
                             device_count=capacity is not None)
    assert np.array_equal(got_v, want_v) and np.array_equal(got_k, want_k)


def test_sort_device_count_and_repeatability():
    rng = np.random.default_rng(9)
    keys = rng.integers(0, 2**40, 123_457, dtype=np.uint64)
    vals = np.arange(keys.size, dtype=np.uint32)
    want_k, want_v = oracle.stable_sort(keys, vals, 0, 40)
    outs = [_gpu_sort(keys, vals, 0, 40, capacity=300_000, device_count=True) for _ in range(3)]
    for got_k, got_v in outs:
        assert np.array_equal(got_k, want_k) and np.array_equal(got_v, want_v)


def test_sort_respects_status_word():
    import torch
    from paper_2602_03207_amd import binding as B
    n = 5000
    kin = torch.arange(n, 0, -1, dtype=torch.int64, device="cuda")
    vin = torch.arange(n, dtype=torch.int32, device="cuda")
    kout = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    vout = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    d_status = torch.tensor([B.WS_ERR_CAPACITY], dtype=torch.int32, device="cuda")
    need = B.ws_sort_workspace_size(n, 0, 32, 0)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    B.ws_sort(kin, vin, kout, vout, n, None, d_status, 0, 32, 0, ws, ws.numel())
    torch.cuda.synchronize()
    assert bool((kout == -1).all()) and bool((vout == -1).all())


def test_sort_oracle_key_buffer_1m_scene():
    """The oracle's own (tile | depth) pair buffer of the 1M-Gaussian 1080p view."""
    scene, cam = scenegen.c2()
    keys, vals = oracle.emit(scene, cam, oracle.Options(sh_degree=3))
    assert keys.size > 1_000_000
    end_bit = 32 + int(np.ceil(np.log2(120 * 68)))
    want_k, want_v = oracle.stable_sort(keys, vals, 0, end_bit)
    for rb in (8, 6):
        got_k, got_v = _gpu_sort(keys, vals, 0, end_bit, rb)
        assert np.array_equal(got_k, want_k) and np.array_equal(got_v, want_v), rb


@pytest.mark.slow
def test_sort_oracle_key_buffer_6m_scene_both_key_widths():
    """The oracle's pair buffer of the 6M-Gaussian 4K view (about 49 M pairs, 12 011 sort tiles of 4096 pairs:
    the digit tables of its passes take the three-level scan), bit-exact against std::stable_sort and identical
    run to run: the 64-bit (tile | depth) sort over the tile and depth bits, and the depth-first variant (pairs
    stably ordered by depth first, then 32-bit tile keys sorted by ws_sort32 on the tile bits)."""
    import torch
    from paper_2602_03207_amd import binding as B
    scene, cam = scenegen.c3()
    keys, vals = oracle.emit(scene, cam, oracle.Options(sh_degree=3))
    n = keys.size
    assert 40_000_000 <= n <= 60_000_000
    tile_bits = int(np.ceil(np.log2(240 * 135)))
    end_bit = 32 + tile_bits
    sort_tiles = -(-n // 4096)
    # the digit table (radix x tiles) of an 8-bit pass is scanned in blocks of 1024 entries: more than 1024
    # blocks take the three-level schedule
    assert 256 * sort_tiles > 1024 * 1024
    want_k, want_v = oracle.stable_sort(keys, vals, 0, end_bit)
    print(f"6M scene: {n} pairs, {sort_tiles} sort tiles", flush=True)
    runs = [_gpu_sort(keys, vals, 0, end_bit, 8) for _ in range(2)]
    for got_k, got_v in runs:
        assert np.array_equal(got_k, want_k) and np.array_equal(got_v, want_v)
    del runs
    # depth-first: the stable depth order of the emitted pairs, then the tile bits alone as 32-bit keys
    dk, dv = oracle.stable_sort(keys, vals, 0, 32)
    del keys, vals
    tiles32 = (dk >> np.uint64(32)).astype(np.uint32)
    del dk
    want_t = (want_k >> np.uint64(32)).astype(np.uint32)
    del want_k
    kin = torch.from_numpy(tiles32.view(np.int32)).cuda()
    vin = torch.from_numpy(dv.view(np.int32)).cuda()
    outs = []
    for rb in (8, 8, 5):
        kout = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        vout = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
        need = B.ws_sort32_workspace_size(n, 0, tile_bits, rb)
        ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
        print(f"ws_sort32 of {n} tile keys, radix {rb}", flush=True)
        B.ws_sort32(kin, vin, kout, vout, n, None, d_status, 0, tile_bits, rb, ws, ws.numel())
        torch.cuda.synchronize()
        assert int(d_status.item()) == 0
        outs.append((kout.cpu().numpy().view(np.uint32), vout.cpu().numpy().view(np.uint32)))
        del kout, vout, ws
    for got_k, got_v in outs:
        # the same lists as the full-key sort (reading A28) ...
        assert np.array_equal(got_k, want_t) and np.array_equal(got_v, want_v)
    # ... and identical bits run to run
    assert np.array_equal(outs[0][1], outs[1][1])
