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
