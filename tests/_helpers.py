"""Shared helpers of the GPU parity tests (oracle side and GPU side kept apart)."""
import numpy as np

import oracle

F32 = lambda x: float(np.float32(x))  # noqa: E731


def oracle_options(tile_w=16, tile_h=16, sh_degree=0, flags=0, bg=(0.0, 0.0, 0.0)):
    """Oracle options holding exactly the fp32 values the GPU library receives."""
    return oracle.Options(tile_w=tile_w, tile_h=tile_h, sh_degree=sh_degree, flags=flags, near_z=F32(0.2),
                          lowpass=F32(0.3), clamp_fov=F32(1.3), alpha_min=F32(1 / 255), alpha_max=F32(0.99),
                          t_min=F32(1e-4), bg=tuple(F32(b) for b in bg))


def gpu_options(tile_w=16, tile_h=16, sh_degree=0, flags=0, radix_bits=0, bg=(0.0, 0.0, 0.0), bin_x=1, bin_y=1):
    from paper_2602_03207_amd import binding as B
    return B.make_options(tile_w=tile_w, tile_h=tile_h, sh_degree=sh_degree, flags=flags, radix_bits=radix_bits,
                          bg=bg, bin_x=bin_x, bin_y=bin_y)


def unpack_splats(splats_f32: np.ndarray):
    """Fields of a [k, 12] float32 view of ws_splat records."""
    s = np.ascontiguousarray(splats_f32, np.float32)
    rect = s[:, 10:12].view(np.uint32)
    return dict(mean2d=s[:, 0:2].T, conic=s[:, 2:5].T, opacity=s[:, 5], rgb=s[:, 6:9].T, depth=s[:, 9],
                rect=np.stack([rect[:, 0] & 0xFFFF, rect[:, 0] >> 16, rect[:, 1] & 0xFFFF, rect[:, 1] >> 16]))


def pack_splats(mean2d, conic, opacity, rgb, depth, pix_rect):
    """[n, 12] float32 ws_splat records from per-component arrays (rect as inclusive x0, x1, y0, y1)."""
    n = np.asarray(opacity).shape[0]
    out = np.zeros((n, 12), np.float32)
    out[:, 0:2] = np.asarray(mean2d, np.float32).T
    out[:, 2:5] = np.asarray(conic, np.float32).T
    out[:, 5] = np.asarray(opacity, np.float32)
    out[:, 6:9] = np.asarray(rgb, np.float32).T
    out[:, 9] = np.asarray(depth, np.float32)
    r = np.asarray(pix_rect).astype(np.int64)
    r = np.clip(r, 0, 65535).astype(np.uint32)
    w = np.zeros((n, 2), np.uint32)
    w[:, 0] = r[0] | (r[1] << 16)
    w[:, 1] = r[2] | (r[3] << 16)
    out[:, 10:12] = w.view(np.float32)
    return out


def assert_image_parity(gpu, ref, tol=2e-4, sel=None):
    """Every pixel of a GPU image [3, H, W] against the oracle's render `ref` (computed with outcomes=True).

    A pixel whose compositing takes no decision within fp32 reach of its threshold has one correct value:
    |gpu - oracle| <= tol per channel.  The others (ref["outcomes"]: alpha_min or t_min tests whose fp64 value
    lies inside the fp32 error bound of the GPU's evaluation) must lie within tol of one of the composites that
    the combinations of those decisions give, or, where there were too many combinations to list, within the
    bound of what those decisions can change.  `sel` ([H, W] bool) restricts the check to the pixels the oracle
    composited (a masked render).  Returns (worst error on single-outcome pixels, fraction of the checked
    pixels with several outcomes)."""
    gpu = np.asarray(gpu, np.float64)
    _, H, W = gpu.shape
    want = np.asarray(ref["rgb"], np.float64)
    oc = ref["outcomes"]
    sel = np.ones((H, W), bool) if sel is None else np.asarray(sel, bool)
    multi = np.zeros(H * W, bool)
    multi[oc["pix"]] = True
    multi = multi.reshape(H, W)
    assert not np.any(multi & ~sel), "outcomes listed for a pixel the oracle did not composite"
    single = sel & ~multi
    err = np.abs(gpu - want)
    worst = float(err[:, single].max()) if single.any() else 0.0
    bad = np.argwhere(single & (err.max(axis=0) > tol))
    assert worst <= tol, f"max |gpu - oracle| = {worst:.3e} on single-outcome pixels, e.g. (y, x) {bad[:5].tolist()}"
    k = oc["pix"].size
    if k:
        g = gpu.reshape(3, -1)[:, oc["pix"]].T  # [k, 3]
        slots = np.arange(oc["rgb"].shape[1])[None, :]
        dist = np.abs(oc["rgb"] - g[:, None, :]).max(axis=2)
        dist = np.where(slots < oc["n_out"][:, None], dist, np.inf).min(axis=1)
        listed = oc["n_out"] > 0
        assert np.all(dist[listed] <= tol), \
            f"{int(np.sum(dist[listed] > tol))} pixels match none of their outcomes (worst {dist[listed].max():.3e})"
        w = want.reshape(3, -1)[:, oc["pix"]].T
        cut = ~listed
        if cut.any():
            dev = np.abs(g[cut] - w[cut]).max(axis=1)
            assert np.all(dev <= oc["bound"][cut] + tol), "a pixel moves beyond the bound of its decisions"
    frac = float(multi[sel].mean()) if sel.any() else 0.0
    return worst, frac
