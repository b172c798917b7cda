"""ws_sort_noalloc (the sort without a workspace argument, whose scratch is a device array inside the
library) against ws_sort on the same inputs: bit-identical outputs on two calls in a row, the second with a
smaller input and another bit range, so the second call runs on the scratch the first one left behind."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _sort_both(keys, vals, begin_bit, end_bit, radix_bits, device_count=False, capacity=None):
    import torch
    from paper_2602_03207_amd import binding as B
    n = keys.size
    cap = capacity or n
    kin = torch.zeros(cap, dtype=torch.int64, device="cuda")
    vin = torch.zeros(cap, dtype=torch.int32, device="cuda")
    kin[:n] = torch.from_numpy(keys.view(np.int64))
    vin[:n] = torch.from_numpy(vals.view(np.int32))
    d_n = torch.tensor([n], dtype=torch.int64, device="cuda") if device_count else None
    outs = []
    for which in ("ws_sort", "ws_sort_noalloc"):
        kout = torch.full((cap,), -1, dtype=torch.int64, device="cuda")
        vout = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
        d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
        size = cap if device_count else n
        print(f"{which}: n {n}, capacity {size}, bits [{begin_bit}, {end_bit}), radix {radix_bits}", flush=True)
        if which == "ws_sort":
            need = B.ws_sort_workspace_size(size, begin_bit, end_bit, radix_bits)
            ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
            B.ws_sort(kin, vin, kout, vout, size, d_n, d_status, begin_bit, end_bit, radix_bits, ws, ws.numel())
        else:
            B.ws_sort_noalloc(kin, vin, kout, vout, size, d_n, d_status, begin_bit, end_bit, radix_bits)
        torch.cuda.synchronize()
        assert int(d_status.item()) == 0
        outs.append((kout[:n].cpu().numpy().view(np.uint64), vout[:n].cpu().numpy().view(np.uint32)))
    return outs


def test_noalloc_sort_equals_ws_sort_on_two_calls():
    rng = np.random.default_rng(77)
    # first call: the largest input the static scratch takes, all 64 key bits, 8-bit digits
    n1 = 1 << 20
    k1 = rng.integers(0, 2**63, n1, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n1, dtype=np.uint64)
    k1[::7] = k1[3]  # runs of equal keys: stability shows in the values
    v1 = np.arange(n1, dtype=np.uint32)
    (a_k, a_v), (b_k, b_v) = _sort_both(k1, v1, 0, 64, 8)
    assert np.array_equal(a_k, b_k) and np.array_equal(a_v, b_v)
    assert np.all(a_k[1:] >= a_k[:-1])
    # second call, smaller, on what the first call left in the scratch: (tile | depth) keys, the tile and
    # depth bits only, 6-bit digits, count read from device memory
    n2 = 123_457
    k2 = (rng.integers(0, 8160, n2, dtype=np.uint64) << np.uint64(32)) | rng.integers(0, 2**31, n2, dtype=np.uint64)
    v2 = rng.integers(0, 2**32, n2, dtype=np.uint64).astype(np.uint32)
    (a_k, a_v), (b_k, b_v) = _sort_both(k2, v2, 0, 45, 6, device_count=True, capacity=200_000)
    assert np.array_equal(a_k, b_k) and np.array_equal(a_v, b_v)


def test_noalloc_sort_rejects_inputs_beyond_its_scratch():
    from paper_2602_03207_amd import binding as B
    lib = B.load()
    vp = __import__("ctypes").c_void_p
    st = lib.ws_sort_noalloc(vp(0x100000), vp(0x200000), vp(0x300000), vp(0x400000), (1 << 20) + 1, None, None,
                             0, 64, 8, None)
    assert st == B.WS_ERR_INVALID_ARGUMENT and "maximum" in lib.ws_last_error().decode()
