"""Multi-view differentiable step: one launch per stage for all views, captured in a HIP graph.

`BatchedStep` runs, for V cameras of uneven resolution at once:
    preprocess (all views) -> sort (device-sized) -> render (all tiles of all
    views) -> backward of the L1 loss against the targets (all views, the loss
    and its gradient formed inside the compositing adjoint, gradients summed
    over views)
without any host synchronisation, so the whole sequence is captured once with
ws_graph_begin / ws_graph_end and replayed with ws_graph_launch.  Pair buffers
are sized from a measured frame with headroom; a replay that would need more
sets the device status word (checked by `check()`), never writes out of bounds.

`PlainStep` is the reference sequence it is compared with: a host loop over
views, each a single-view forward (with its pair-count read-back), loss (each
view's share of the batch mean) and backward, whose gradients the library adds
to the batch's.

`BatchedForward` / `PlainForward` are the forward-only counterparts (many
views rendered by one captured graph vs one view per launch sequence).
"""
from __future__ import annotations

import torch

from . import binding as B
from .pipeline import GaussianTensors, Renderer


def _zero_grads(g: GaussianTensors):
    return dict(means=torch.zeros_like(g.means), log_scales=torch.zeros_like(g.log_scales),
                quats=torch.zeros_like(g.quats), opacity_logits=torch.zeros_like(g.opacity_logits),
                sh=torch.zeros_like(g.sh))


class BatchedStep:
    def __init__(self, cams, opts: B.ws_options, g: GaussianTensors, targets: torch.Tensor, headroom=1.25,
                 device="cuda"):
        self.g = g
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self.r = Renderer(cams, opts, device=device)
        self.targets = targets.contiguous()
        assert self.targets.numel() == self.r.image_floats
        with torch.cuda.stream(self.stream):
            m = self.r.forward(g, stream=self.stream)  # measure M once, eagerly
            self.r._ensure_capacity(int(m * headroom) + 4096)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.grads = _zero_grads(g)
        self.graph = None
        # one eager step sizes every workspace before any capture
        self.step_eager()
        self.stream.synchronize()

    def step_eager(self):
        s = self.stream
        with torch.cuda.stream(s):
            self.r.forward_capacity(self.g, stream=s)
            # the L1 loss and its gradient are formed inside the compositing adjoint
            self.r.backward_l1(self.g, self.targets, self.loss, grads=self.grads, stream=s)

    def capture(self):
        s = self.stream
        s.synchronize()
        B.ws_graph_begin(s)
        try:
            self.step_eager()
        except Exception:
            B.ws_graph_end(s)
            raise
        self.graph = B.ws_graph_end(s)

    def replay(self):
        if self.graph is None:
            self.capture()
        B.ws_graph_launch(self.graph, self.stream)

    def check(self):
        self.stream.synchronize()
        st = self.r.status()
        if st != 0:
            raise B.WsError(st, B.ws_status_string(st))

    def close(self):
        if self.graph is not None:
            B.ws_graph_destroy(self.graph)
            self.graph = None


class PlainStep:
    """One view per launch sequence: per view forward (M read back), L1 loss, backward."""

    def __init__(self, cams, opts: B.ws_options, g: GaussianTensors, targets: torch.Tensor, device="cuda"):
        self.g = g
        self.cams = list(cams)
        self.renderers = [Renderer([c], opts, device=device) for c in self.cams]
        sizes = [r.image_floats for r in self.renderers]
        self.targets = list(torch.split(targets.contiguous(), sizes))
        self.total = sum(sizes)
        self.dL = [torch.empty(sz, dtype=torch.float32, device=device) for sz in sizes]
        self.loss = torch.zeros(len(self.cams), dtype=torch.float32, device=device)
        self.ws_loss = torch.empty(max(B.ws_l1_loss_workspace_size(max(sizes)), 256), dtype=torch.uint8,
                                   device=device)
        self.grads = _zero_grads(g)

    def step(self, stream=None):
        for k in self.grads:
            self.grads[k].zero_()
        for v, r in enumerate(self.renderers):
            r.forward(self.g, stream=stream)
            # each view's share of the batch loss (the mean over every view's elements)
            B.ws_l1_loss(r.images, self.targets[v], r.image_floats, self.total, self.dL[v], self.loss[v:v + 1],
                         self.ws_loss, self.ws_loss.numel(), stream)
            # the library adds each view's gradients to the batch's (WS_FLAG_ACCUMULATE_GRADS)
            r.backward(self.g, self.dL[v], grads=self.grads, stream=stream, accumulate=True)
        return self.grads

    def images(self):
        return torch.cat([r.images for r in self.renderers])


class BatchedForward:
    """All views' forward (preprocess, device-sized sort, render) as one graph replay."""

    def __init__(self, cams, opts: B.ws_options, g: GaussianTensors, headroom=1.1, device="cuda"):
        self.g = g
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self.r = Renderer(cams, opts, device=device)
        with torch.cuda.stream(self.stream):
            m = self.r.forward(g, stream=self.stream)
            self.r._ensure_capacity(int(m * headroom) + 4096)
            self.r.forward_capacity(g, stream=self.stream)  # sizes the workspaces at this capacity
        self.stream.synchronize()
        self.graph = None

    def capture(self):
        s = self.stream
        s.synchronize()
        B.ws_graph_begin(s)
        try:
            with torch.cuda.stream(s):
                self.r.forward_capacity(self.g, stream=s)
        except Exception:
            B.ws_graph_end(s)
            raise
        self.graph = B.ws_graph_end(s)

    def replay(self):
        if self.graph is None:
            self.capture()
        B.ws_graph_launch(self.graph, self.stream)

    def check(self):
        self.stream.synchronize()
        st = self.r.status()
        if st != 0:
            raise B.WsError(st, B.ws_status_string(st))

    def close(self):
        if self.graph is not None:
            B.ws_graph_destroy(self.graph)
            self.graph = None


class PlainForward:
    """One view per launch sequence, each with its pair-count read-back."""

    def __init__(self, cams, opts: B.ws_options, g: GaussianTensors, device="cuda"):
        self.g = g
        self.renderers = [Renderer([c], opts, device=device) for c in cams]

    def step(self, stream=None):
        for r in self.renderers:
            r.forward(self.g, stream=stream)

    def images(self):
        return torch.cat([r.images for r in self.renderers])
