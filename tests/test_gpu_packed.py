"""WS_FLAG_PACKED (Sec. 3.2's packed render inputs: fp16 ellipse axes, RGBA8 colour and opacity in 32-byte
records) against the oracle's packed mode: the records field by field, images at the quantisation bound, and
the same images from every layout (tile keys, bins, 32-bit keys)."""
import numpy as np
import pytest

import oracle
import scenegen
from _helpers import assert_image_parity, gpu_options, oracle_options

pytestmark = pytest.mark.gpu

Q = 1.0 / 255.0  # one step of the RGBA8 quantisation


def _scene():
    # SH degree 1 with a wide DC spread: some colours exceed 1 and are clamped by the packing
    return scenegen.random_scene(5000, 61, mean_lo=-1.3, mean_hi=1.3, log_scale_mu=-3.2, logit_sd=2.0, sh_degree=1,
                                 dc_sd=1.0, rest_sd=0.3)


def _render(scene, cams, **kw):
    import torch
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    r = Renderer(cams, gpu_options(sh_degree=scene.sh_degree, **kw))
    r.forward(GaussianTensors.from_scene(scene))
    torch.cuda.synchronize()
    return r


def test_packed_records_match_the_oracle_packing():
    from paper_2602_03207_amd import binding as B
    scene = _scene()
    cam = scenegen.look_at([0.4, -0.2, -3.0], [0, 0, 0], 200, 150)
    r = _render(scene, [cam], flags=B.WS_FLAG_PACKED)
    proj = oracle.preprocess(scene, cam, oracle_options(sh_degree=1))
    tt = r.tiles_touched.cpu().numpy()
    vis = proj["status"] == 0
    assert np.array_equal(tt != 0, vis)
    rec = r.splats.cpu().numpy()[:scene.n]  # [n, 8] float32 words
    words = rec.view(np.uint32)
    idx = np.nonzero(vis)[0]
    # centre and depth as in the full record; rectangle exact
    assert np.allclose(rec[idx, 0:2].T, proj["mean2d"][:, idx], rtol=2e-6, atol=1e-4)
    assert np.array_equal(rec[idx, 5], proj["depth32"][idx])
    rect = np.stack([words[idx, 6] & 0xFFFF, words[idx, 6] >> 16, words[idx, 7] & 0xFFFF, words[idx, 7] >> 16])
    assert np.array_equal(rect, proj["pix_rect"][:, idx])
    # fp16 axes: equal to the oracle's axes rounded to fp16 almost everywhere; where an ellipse is nearly round
    # its eigenvectors turn with any rounding of its covariance, so the ellipse the axes rebuild is compared:
    # within a few fp16 steps of the largest eigenvalue
    want_ax = oracle.ellipse_axes(proj["cov2d"][:, idx]).astype(np.float16).astype(np.float64)
    got_ax = np.stack([(words[idx, 2] & 0xFFFF).astype(np.uint16), (words[idx, 2] >> 16).astype(np.uint16),
                       (words[idx, 3] & 0xFFFF).astype(np.uint16), (words[idx, 3] >> 16).astype(np.uint16)]
                      ).view(np.float16).astype(np.float64)
    diff = np.abs(got_ax - want_ax)
    assert np.mean(np.all(diff == 0, axis=0)) >= 0.99

    def ellipse(ax):
        return np.stack([ax[0] ** 2 + ax[2] ** 2, ax[0] * ax[1] + ax[2] * ax[3], ax[1] ** 2 + ax[3] ** 2])

    lam1 = want_ax[0] ** 2 + want_ax[1] ** 2
    dev = np.abs(ellipse(got_ax) - ellipse(want_ax)) / lam1[None]
    assert np.all(dev <= 4 * 2.0 ** -10), float(dev.max())
    # RGBA8: one step apart at most, and equal almost everywhere (fp32 vs fp64 values at a rounding boundary)
    _, op_q, rgb_q = oracle.pack_quantise(proj)
    want = np.vstack([np.rint(rgb_q[:, idx] * 255), np.rint(op_q[idx] * 255)[None]]).astype(np.int64)
    got = np.stack([(words[idx, 4] >> s) & 0xFF for s in (0, 8, 16, 24)]).astype(np.int64)
    assert np.all(np.abs(got - want) <= 1) and np.mean(got == want) >= 0.999
    print(f"{idx.size} packed records: fp16 axes equal on {np.mean(diff == 0):.5f}, bytes on {np.mean(got == want):.5f}")


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 16)])
def test_packed_image_at_the_quantisation_bound(tile):
    from paper_2602_03207_amd import binding as B
    scene = _scene()
    cam = scenegen.look_at([0.4, -0.2, -3.0], [0, 0, 0], 200, 150)
    r = _render(scene, [cam], tile_w=tile[0], tile_h=tile[1], flags=B.WS_FLAG_PACKED)
    ref = oracle.render(scene, cam, oracle_options(*tile, sh_degree=1), packed=True, outcomes=True)
    assert r.num_pairs == ref["keys"].size
    img = r.image(0).cpu().numpy()
    # every pixel within one quantisation step; pixels where GPU and oracle quantised every input alike agree
    # to the image tolerance, so the pixels beyond it are few
    worst, frac = assert_image_parity(img, ref, tol=Q + 1e-5)
    err = np.abs(img - ref["rgb"]).max(axis=0)
    beyond = float(np.mean(err > 2e-4))
    print(f"packed {tile}: worst {worst:.2e}, {beyond:.2e} of pixels beyond 2e-4, {frac:.2e} with several outcomes")
    assert beyond <= 2e-3


def test_packed_images_identical_across_layouts():
    from paper_2602_03207_amd import binding as B
    scene = _scene()
    cams = [scenegen.look_at([0.4, -0.2, -3.0], [0, 0, 0], 200, 150),
            scenegen.look_at([-1.5, 0.4, -2.4], [0, 0, 0], 97, 131)]
    base = _render(scene, cams, flags=B.WS_FLAG_PACKED).images.cpu().numpy()
    df = B.WS_FLAG_PACKED | B.WS_FLAG_DEPTH_FIRST
    for kw in (dict(flags=df), dict(flags=df | B.WS_FLAG_KEYS32), dict(flags=df | B.WS_FLAG_KEYS32, bin_x=4, bin_y=2),
               dict(flags=B.WS_FLAG_PACKED, bin_x=2, bin_y=2), dict(flags=df | B.WS_FLAG_KEYS32, bin_x=8, bin_y=8),
               dict(flags=B.WS_FLAG_PACKED | B.WS_FLAG_ORDERED_RENDER)):
        img = _render(scene, cams, **kw).images.cpu().numpy()
        assert np.array_equal(img.view(np.uint32), base.view(np.uint32)), kw


@pytest.mark.slow
def test_packed_c2_frame_at_the_quantisation_bound():
    """The 1M-Gaussian 1080p view in the benchmark layout with packed records, against the oracle's packing."""
    import torch
    from paper_2602_03207_amd import binding as B
    from paper_2602_03207_amd.batched import BatchedForward
    from paper_2602_03207_amd.pipeline import GaussianTensors
    scene, cam = scenegen.c2()
    opts = gpu_options(sh_degree=3, bin_x=4, bin_y=2, flags=B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32 | B.WS_FLAG_PACKED)
    bf = BatchedForward([cam], opts, GaussianTensors.from_scene(scene))
    bf.capture()
    bf.replay()
    bf.check()
    torch.cuda.synchronize()
    img = bf.r.image(0).cpu().numpy()
    bf.close()
    ref = oracle.render(scene, cam, oracle_options(sh_degree=3), packed=True, outcomes=True)
    worst, frac = assert_image_parity(img, ref, tol=Q + 1e-5)
    beyond = float(np.mean(np.abs(img - ref["rgb"]).max(axis=0) > 2e-4))
    print(f"packed C2: worst {worst:.2e}, {beyond:.2e} of pixels beyond 2e-4")
    assert beyond <= 2e-3
