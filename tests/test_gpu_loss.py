"""The L1 loss of the training step (ws_l1_loss) against the oracle's L1 (reading A19: the mean over every
element of the batch, sign(0) = 0), the gradient accumulation of ws_render_backward, and the status checks
of the plain path (a device status word set from the host: every kernel then exits at once)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _pair(rng, n, equal_frac=0.05):
    img = rng.random(n, dtype=np.float32)
    tgt = (img + rng.normal(0, 0.2, n)).astype(np.float32)
    eq = rng.random(n) < equal_frac
    tgt[eq] = img[eq]  # sign(0) = 0 on these
    return img, tgt


def _gpu_l1(parts_img, parts_tgt, total):
    import torch
    from paper_2602_03207_amd import binding as B
    losses, grads = [], []
    ws = torch.empty(max(B.ws_l1_loss_workspace_size(max(p.size for p in parts_img)), 256), dtype=torch.uint8,
                     device="cuda")
    for img, tgt in zip(parts_img, parts_tgt):
        di, dt = torch.from_numpy(img).cuda(), torch.from_numpy(tgt).cuda()
        dL = torch.full_like(di, 7.0)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        B.ws_l1_loss(di, dt, di.numel(), total, dL, loss, ws, ws.numel())
        torch.cuda.synchronize()
        losses.append(float(loss.item()))
        grads.append(dL.cpu().numpy())
    return losses, grads


def test_l1_loss_matches_oracle_1080p():
    rng = np.random.default_rng(31)
    n = 3 * 1080 * 1920
    img, tgt = _pair(rng, n)
    want_loss, want_g = oracle.l1_loss_grad(img, tgt)
    (loss,), (g,) = _gpu_l1([img], [tgt], 0)
    print(f"1080p L1: gpu {loss!r} oracle {want_loss!r}")
    assert abs(loss - want_loss) <= 1e-6 * want_loss
    # every gradient element is sign / numel rounded once to fp32
    assert np.array_equal(g, want_g.astype(np.float32))
    assert np.count_nonzero(g == 0) == np.count_nonzero(img == tgt) > 0


def test_l1_loss_split_over_views_is_the_batch_loss():
    """Views of uneven size, one call each with the batch's element count: the per-call losses add up to
    the batch loss and each gradient is that of the batch loss."""
    rng = np.random.default_rng(32)
    sizes = [3 * 512 * 512, 3 * 720 * 1280, 3 * 61 * 77]
    pairs = [_pair(rng, s) for s in sizes]
    imgs, tgts = [p[0] for p in pairs], [p[1] for p in pairs]
    want_loss, want_g = oracle.l1_loss_grad(imgs, tgts)
    losses, grads = _gpu_l1(imgs, tgts, sum(sizes))
    assert abs(sum(losses) - want_loss) <= 1e-6 * want_loss
    for g, w in zip(grads, want_g):
        assert np.array_equal(g, w.astype(np.float32))


def test_accumulate_flag_adds_to_the_gradients():
    import torch
    import scenegen
    from _helpers import gpu_options
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    scene = scenegen.random_scene(1500, 21, sh_degree=1, dc_sd=0.4, rest_sd=0.2)
    cam = scenegen.look_at([0.2, 0.1, -3.0], [0, 0, 0], 80, 64)
    g = GaussianTensors.from_scene(scene)
    r = Renderer([cam], gpu_options(sh_degree=1))
    r.forward(g)
    dL = torch.randn_like(r.images)
    fresh = r.backward(g, dL, check=True)
    base = {k: torch.randn_like(v) for k, v in fresh.items()}
    acc = {k: v.clone() for k, v in base.items()}
    r.backward(g, dL, grads=acc, accumulate=True, check=True)
    for k in fresh:
        want = base[k].double() + fresh[k].double()
        scale = want.abs().max().item()
        # the two backward calls differ only in the order of their floating-point atomic additions
        assert torch.allclose(acc[k].double(), want, rtol=1e-5, atol=1e-6 * scale), k


def test_backward_writes_nothing_and_raises_when_the_forward_failed():
    import torch
    import scenegen
    from _helpers import gpu_options
    from paper_2602_03207_amd import binding as B
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    scene = scenegen.random_scene(800, 22, sh_degree=0)
    cam = scenegen.look_at([0.0, 0.0, -3.0], [0, 0, 0], 64, 48)
    g = GaussianTensors.from_scene(scene)
    r = Renderer([cam], gpu_options())
    r.forward(g)
    grads = {k: torch.full_like(getattr(g, k), 5.0) for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
    r.d_status.fill_(B.WS_ERR_SPIN_LIMIT)  # as a sort whose bounded wait expired would leave it
    with pytest.raises(B.WsError):
        r.backward(g, torch.ones_like(r.images), grads=grads, check=True)
    for k, v in grads.items():
        assert torch.all(v == 5.0), k


def test_forward_raises_when_a_late_stage_failed(monkeypatch):
    """The plain forward reads the status word again after the render: a failure reported by the sort or
    the render (here written from the host after the render) raises instead of returning stale images."""
    import scenegen
    from _helpers import gpu_options
    from paper_2602_03207_amd import binding as B
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    scene = scenegen.random_scene(800, 23, sh_degree=0)
    cam = scenegen.look_at([0.0, 0.0, -3.0], [0, 0, 0], 64, 48)
    g = GaussianTensors.from_scene(scene)
    r = Renderer([cam], gpu_options())
    r.forward(g)
    orig = Renderer.render

    def failing_render(self, cap, stream=None):
        orig(self, cap, stream)
        self.d_status.fill_(B.WS_ERR_SPIN_LIMIT)

    monkeypatch.setattr(Renderer, "render", failing_render)
    with pytest.raises(B.WsError):
        r.forward(g)


def _fused_vs_separate(scene, cams, opts, tgt_scene, total=0):
    """ws_render_backward_l1 against ws_l1_loss + ws_render_backward on the same forward."""
    import torch
    from paper_2602_03207_amd import binding as B
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    g = GaussianTensors.from_scene(scene)
    tr = Renderer(cams, opts)
    tr.forward(GaussianTensors.from_scene(tgt_scene))
    targets = tr.images.clone()
    r = Renderer(cams, opts)
    r.forward(g)
    n = r.image_floats
    dL = torch.empty_like(r.images)
    loss_sep = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = torch.empty(max(B.ws_l1_loss_workspace_size(n), 256), dtype=torch.uint8, device="cuda")
    B.ws_l1_loss(r.images, targets, n, total, dL, loss_sep, ws, ws.numel())
    sep = r.backward(g, dL, check=True)
    loss_fused = torch.full((1,), -1.0, dtype=torch.float32, device="cuda")
    fused = r.backward_l1(g, targets, loss_fused, total=total, check=True)
    torch.cuda.synchronize()
    return r, targets, float(loss_sep.item()), float(loss_fused.item()), sep, fused


@pytest.mark.parametrize("views,bins", [(1, (1, 1)), (3, (4, 2))])
def test_fused_l1_backward_equals_loss_then_backward(views, bins):
    """ws_render_backward_l1 forms dL/dC = sign(image - target) / total inside the adjoint: its gradients are
    those of ws_l1_loss followed by ws_render_backward (up to the order of the floating-point atomics), and
    its loss is the oracle's L1 of the same images (fp64 sums in another order, rounded once)."""
    import scenegen
    from _helpers import gpu_options
    from paper_2602_03207_amd import binding as B
    scene = scenegen.random_scene(3000, 41, sh_degree=2, dc_sd=0.4, rest_sd=0.2)
    tgt_scene = scenegen.random_scene(3000, 42, sh_degree=2, dc_sd=0.4, rest_sd=0.2)
    cams = [scenegen.look_at([0.3 * v - 0.3, 0.1, -3.0], [0, 0, 0], 96 + 17 * v, 72 + 9 * v) for v in range(views)]
    flags = B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_KEYS32
    opts = gpu_options(sh_degree=2, flags=flags, bin_x=bins[0], bin_y=bins[1])
    r, targets, loss_sep, loss_fused, sep, fused = _fused_vs_separate(scene, cams, opts, tgt_scene)
    img, tgt = r.images.cpu().numpy(), targets.cpu().numpy()
    want_loss, _ = oracle.l1_loss_grad(img, tgt)
    print(f"views {views}: fused {loss_fused!r} separate {loss_sep!r} oracle {want_loss!r}")
    assert abs(loss_fused - want_loss) <= 1e-6 * want_loss
    assert abs(loss_fused - loss_sep) <= 2 * np.spacing(np.float32(want_loss))
    for k in sep:
        a, b = sep[k].double(), fused[k].double()
        scale = a.abs().max().item()
        assert scale > 0, k
        assert float((a - b).abs().max()) <= 1e-5 * scale, k


def test_fused_l1_backward_batch_total_and_status():
    """A `total` larger than the views' elements scales the loss and every gradient by elements / total; a set
    status word leaves gradients and loss untouched."""
    import torch
    import scenegen
    from _helpers import gpu_options
    from paper_2602_03207_amd import binding as B
    scene = scenegen.random_scene(1200, 43, sh_degree=1, dc_sd=0.4, rest_sd=0.2)
    tgt_scene = scenegen.random_scene(1200, 44, sh_degree=1, dc_sd=0.4, rest_sd=0.2)
    cams = [scenegen.look_at([0.0, 0.2, -3.0], [0, 0, 0], 80, 64)]
    opts = gpu_options(sh_degree=1)
    elems = 3 * 80 * 64
    r, targets, _, loss1, _, g1 = _fused_vs_separate(scene, cams, opts, tgt_scene)
    loss4 = torch.zeros(1, dtype=torch.float32, device="cuda")
    from paper_2602_03207_amd.pipeline import GaussianTensors
    g = GaussianTensors.from_scene(scene)
    g4 = r.backward_l1(g, targets, loss4, total=4 * elems, check=True)
    torch.cuda.synchronize()
    assert abs(float(loss4.item()) * 4 - loss1) <= 1e-6 * loss1
    for k in g1:
        a, b = g1[k].double(), 4 * g4[k].double()
        assert float((a - b).abs().max()) <= 1e-5 * a.abs().max().item(), k
    grads = {k: torch.full_like(v, 5.0) for k, v in g1.items()}
    loss = torch.full((1,), -3.0, dtype=torch.float32, device="cuda")
    r.d_status.fill_(B.WS_ERR_SPIN_LIMIT)
    with pytest.raises(B.WsError):
        r.backward_l1(g, targets, loss, grads=grads, check=True)
    assert float(loss.item()) == -3.0
    for k, v in grads.items():
        assert torch.all(v == 5.0), k
