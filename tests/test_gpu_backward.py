"""ws_render_backward on the GPU against the fp64 oracle's reverse mode; autograd and batched/graph paths."""
import numpy as np
import pytest

import oracle
import scenegen
from _helpers import gpu_options, oracle_options

pytestmark = pytest.mark.gpu

NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _gpu_grads(scene, cams, dL_views, **kw):
    import torch
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    r = Renderer(cams, gpu_options(sh_degree=scene.sh_degree, **kw))
    g = GaussianTensors.from_scene(scene)
    r.forward(g)
    dL = torch.as_tensor(np.concatenate([np.asarray(d, np.float32).reshape(-1) for d in dL_views])).cuda()
    grads = r.backward(g, dL)
    torch.cuda.synchronize()
    assert r.status() == 0
    return {k: grads[k].cpu().numpy().astype(np.float64) for k in NAMES}, r


def _oracle_grads(scene, cams, dL_views, ropts):
    tot = {k: 0.0 for k in NAMES}
    for cam, dL in zip(cams, dL_views):
        res = oracle.forward_backward(scene, cam, ropts, np.asarray(dL, np.float32).astype(np.float64))
        for k in NAMES:
            tot[k] = tot[k] + res["grads"][k]
    return tot


def _compare(got, want, rel=1e-3, elem_frac=0.999, outlier_rel=1e-2):
    """Reading A24: per tensor ||g - g*|| / ||g*|| <= rel; per element |g - g*| <= rel * max(|g*|, rms g*) on at
    least elem_frac of the elements, and every element within outlier_rel of that scale (the remaining elements
    are those of splats with a decision near its threshold at some pixel, where fp32 and fp64 may differ)."""
    for k in NAMES:
        g, w = got[k].reshape(-1), want[k].reshape(-1)
        nrm = np.linalg.norm(w)
        if nrm == 0:
            assert np.linalg.norm(g) == 0, k
            continue
        err = np.linalg.norm(g - w) / nrm
        assert err <= rel, f"{k}: relative error {err:.2e}"
        scale = np.maximum(np.abs(w), np.sqrt(np.mean(w * w)))
        ratio = np.abs(g - w) / scale
        ok = ratio <= rel
        worst = int(np.argmax(ratio))
        print(f"{k}: norm error {err:.2e}, {np.count_nonzero(~ok)} of {ok.size} elements above {rel:g}, worst "
              f"element {worst}: {ratio[worst]:.2e} of its scale (gpu {g[worst]:.6e}, oracle {w[worst]:.6e})")
        assert ok.mean() >= elem_frac, f"{k}: {np.count_nonzero(~ok)} of {ok.size} elements off"
        assert ratio[worst] <= outlier_rel, f"{k}: element {worst} off by {ratio[worst]:.2e} of its scale"


def test_backward_fd_scene_matches_oracle():
    scene, cam = scenegen.fd_scene()
    rng = np.random.default_rng(3)
    dL = rng.standard_normal((3, cam.height, cam.width)).astype(np.float32)
    got, _ = _gpu_grads(scene, [cam], [dL])
    want = _oracle_grads(scene, [cam], [dL], oracle_options(sh_degree=3))
    _compare(got, want)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 16)])
def test_backward_multiview_matches_oracle(tile):
    scene = scenegen.random_scene(2500, 8, log_scale_mu=-3.0, logit_sd=2.0, sh_degree=1, dc_sd=0.5, rest_sd=0.2)
    cams = [scenegen.look_at([0.3, -0.2, -3.0], [0, 0, 0], 128, 96), scenegen.look_at([2.0, 0.5, -2.0], [0, 0, 0], 77, 61),
            scenegen.look_at([-1.0, -1.5, -2.0], [0, 0, 0], 100, 100)]
    rng = np.random.default_rng(4)
    dLs = [rng.standard_normal((3, c.height, c.width)).astype(np.float32) for c in cams]
    got, _ = _gpu_grads(scene, cams, dLs, tile_w=tile[0], tile_h=tile[1])
    want = _oracle_grads(scene, cams, dLs, oracle_options(*tile, sh_degree=1))
    _compare(got, want)


@pytest.mark.parametrize("deg", [0, 2])
def test_backward_sh_degrees_match_oracle(deg):
    """The geometry and colour adjoint kernels at the SH degrees the other tests leave out, two views
    (the colour kernel sums the view directions' gradients into the means)."""
    scene = scenegen.random_scene(2000, 12 + deg, log_scale_mu=-3.0, logit_sd=2.0, sh_degree=deg, dc_sd=0.5,
                                  rest_sd=0.2)
    cams = [scenegen.look_at([0.4, 0.3, -3.0], [0, 0, 0], 96, 80), scenegen.look_at([-1.8, 0.2, -2.2], [0, 0, 0], 90, 72)]
    rng = np.random.default_rng(20 + deg)
    dLs = [rng.standard_normal((3, c.height, c.width)).astype(np.float32) for c in cams]
    got, _ = _gpu_grads(scene, cams, dLs)
    want = _oracle_grads(scene, cams, dLs, oracle_options(sh_degree=deg))
    _compare(got, want)


@pytest.mark.slow
def test_backward_1080p_l1_view_matches_oracle():
    """One 1920x1080 view of the 1M-Gaussian scene with the L1 loss against a perturbed-scene target, with
    tile keys and in the training benchmark's layout (16x16 tiles in 4x2 bins, 32-bit keys)."""
    from paper_2602_03207_amd import binding as B
    scene, cams, target_scene = scenegen.c5(n_views=1)
    cam = cams[0]
    ro = oracle_options(sh_degree=3)
    img = oracle.forward_backward(scene, cam, ro)["image"]
    tgt = oracle.forward_backward(target_scene, cam, ro)["image"]
    _, dL = oracle.l1_loss_grad(img, tgt)
    dL = dL.astype(np.float32)
    want = _oracle_grads(scene, [cam], [dL], ro)
    for kw in ({}, dict(bin_x=4, bin_y=2, flags=B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32)):
        print(f"1080p backward, options {kw}", flush=True)
        got, _ = _gpu_grads(scene, [cam], [dL], **kw)
        _compare(got, want)


@pytest.mark.parametrize("bins", [(4, 2), (2, 2)])
def test_backward_binned_32bit_keys_match_oracle(bins):
    """The training benchmark's layout (16x16 tiles in bins, 32-bit keys, depth-first emission): the
    backward reads the expanded per-tile lists; three views of uneven size against the oracle."""
    from paper_2602_03207_amd import binding as B
    scene = scenegen.random_scene(2500, 8, log_scale_mu=-3.0, logit_sd=2.0, sh_degree=1, dc_sd=0.5, rest_sd=0.2)
    cams = [scenegen.look_at([0.3, -0.2, -3.0], [0, 0, 0], 128, 96), scenegen.look_at([2.0, 0.5, -2.0], [0, 0, 0], 77, 61),
            scenegen.look_at([-1.0, -1.5, -2.0], [0, 0, 0], 100, 100)]
    rng = np.random.default_rng(5)
    dLs = [rng.standard_normal((3, c.height, c.width)).astype(np.float32) for c in cams]
    got, _ = _gpu_grads(scene, cams, dLs, bin_x=bins[0], bin_y=bins[1],
                        flags=B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32)
    want = _oracle_grads(scene, cams, dLs, oracle_options(sh_degree=1))
    _compare(got, want)


def test_backward_tile_counts_gate_the_gradient_records():
    """With ws_preprocess's tile counts the adjoint clears and reads only the gradient records of entries in
    some tile list; without them (NULL) every record.  Both start from a workspace of NaN bytes: the records
    the counts skip are never read, and both calls give the same gradients (up to the order of the float
    atomics) as the oracle."""
    import torch
    from paper_2602_03207_amd import binding as B
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    scene = scenegen.random_scene(2500, 8, log_scale_mu=-3.0, logit_sd=2.0, sh_degree=1, dc_sd=0.5, rest_sd=0.2)
    cams = [scenegen.look_at([0.3, -0.2, -3.0], [0, 0, 0], 128, 96), scenegen.look_at([2.0, 0.5, -2.0], [0, 0, 0], 77, 61)]
    rng = np.random.default_rng(6)
    dLs = [rng.standard_normal((3, c.height, c.width)).astype(np.float32) for c in cams]
    r = Renderer(cams, gpu_options(sh_degree=1))
    g = GaussianTensors.from_scene(scene)
    r.forward(g)
    assert int((r.tiles_touched[:len(cams) * g.n] == 0).sum()) > 0  # some entries are culled
    dL = torch.as_tensor(np.concatenate([d.reshape(-1) for d in dLs])).cuda()
    need = B.ws_render_backward_workspace_size(g.n, len(cams))
    out = []
    for touched in (r.tiles_touched, None):
        ws = torch.full((need + 256,), 0xFF, dtype=torch.uint8, device="cuda")
        off = (-ws.data_ptr()) % 256
        ws = ws[off:off + need]
        grads = {k: torch.zeros_like(getattr(g, k)) for k in NAMES}
        gs = B.make_grads(grads["means"], grads["log_scales"], grads["quats"], grads["opacity_logits"], grads["sh"])
        B.ws_render_backward(g.struct(), r.cam_arr, r.d_cams, r.n_views, r.opts, r.splats, touched, r.lists,
                             r.tile_ranges, r.images, dL, r.d_status, gs, ws, need)
        torch.cuda.synchronize()
        assert r.status() == 0
        out.append({k: grads[k].cpu().numpy().astype(np.float64) for k in NAMES})
    for k in NAMES:
        assert np.isfinite(out[0][k]).all() and np.isfinite(out[1][k]).all(), k
        np.testing.assert_allclose(out[0][k], out[1][k], rtol=1e-4, atol=1e-6 * np.abs(out[1][k]).max(), err_msg=k)
    _compare(out[0], _oracle_grads(scene, cams, dLs, oracle_options(sh_degree=1)))


def test_autograd_function_matches_backward_call():
    import torch
    from paper_2602_03207_amd.autograd import render_gaussians
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    scene = scenegen.random_scene(1500, 9, sh_degree=2, dc_sd=0.4, rest_sd=0.2)
    cam = scenegen.look_at([0.1, 0.2, -3.0], [0, 0, 0], 96, 72)
    g = GaussianTensors.from_scene(scene)
    params = [getattr(g, k).clone().requires_grad_(True) for k in NAMES]
    r = Renderer([cam], gpu_options(sh_degree=2))
    img = render_gaussians(*params, r)
    w = torch.randn_like(img)
    (img * w).sum().backward()
    r2 = Renderer([cam], gpu_options(sh_degree=2))
    r2.forward(g)
    assert torch.equal(r2.images, img.detach())
    ref = r2.backward(g, w)
    for k, p in zip(NAMES, params):
        # the two backward calls differ only in the order of their floating-point atomic additions
        rms = ref[k].double().pow(2).mean().sqrt().item()
        assert torch.allclose(p.grad, ref[k], rtol=1e-4, atol=1e-5 * rms), k


@pytest.mark.parametrize("layout", ["tile_keys", "bench"])
def test_batched_graph_equals_plain_and_replays_consistently(layout):
    import torch
    from paper_2602_03207_amd import binding as B
    from paper_2602_03207_amd.batched import BatchedStep, PlainStep
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    scene = scenegen.random_scene(4000, 10, log_scale_mu=-3.2, sh_degree=3, dc_sd=0.5, rest_sd=0.2)
    target = scenegen.perturb(scene, 99)
    rng = np.random.default_rng(1)
    res = [(128, 128), (160, 90), (96, 120), (200, 64)]
    cams = scenegen.orbit_cameras(rng, len(res), res)
    opts = gpu_options(sh_degree=3) if layout == "tile_keys" else \
        gpu_options(sh_degree=3, bin_x=4, bin_y=2, flags=B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32)
    g = GaussianTensors.from_scene(scene)
    tr = Renderer(cams, opts)
    tr.forward(GaussianTensors.from_scene(target))
    targets = tr.images.clone()
    plain = PlainStep(cams, opts, g, targets)
    pg = {k: v.clone() for k, v in plain.step().items()}
    pimg = plain.images().clone()
    bs = BatchedStep(cams, opts, g, targets)
    bs.capture()
    for rep in range(3):
        with torch.cuda.stream(bs.stream):  # eager work between replays; the graph must overwrite it
            for k in bs.grads:
                bs.grads[k].fill_(123.0)
            bs.r.images.fill_(-1.0)
        bs.replay()
        bs.check()
        assert torch.equal(bs.r.images, pimg), rep
        for k in NAMES:
            a, b = bs.grads[k].double(), pg[k].double()
            err = (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item()
            assert err <= 1e-3, (rep, k, err)
    bs.close()
