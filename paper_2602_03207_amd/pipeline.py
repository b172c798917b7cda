"""Buffers and call sequences of the render path on one GPU.

`Renderer` owns the device buffers and workspaces and issues the C calls in
order; it never computes anything itself.  Two sequences are provided:

* plain (`forward`): preprocess, read the pair count M back to the host,
  sort exactly M pairs, render.  One host synchronisation per frame.
* device-sized (`forward_capacity`): the sort and the render read M from
  device memory and are launched for the preallocated capacity, so the
  whole frame (and a backward) can be captured in a HIP graph.

With WS_FLAG_KEYS32 (depth-first emission only) the keys are 32-bit tile
ids and the sort is `ws_sort32` over the tile bits.

With bins larger than one tile (options bin_x, bin_y) the pairs name bins:
the sort orders the bin bits, and `ws_expand_bins` builds every tile's list
(in `tile_vals`, one slot per tile of the bin's pair count) and the tile
ranges that the render and the backward read.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import binding as B


@dataclass
class GaussianTensors:
    """Device copies of the Gaussian parameters (fp32, component-major)."""
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacity_logits: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    def struct(self) -> B.ws_gaussians:
        return B.make_gaussians(self.n, self.means, self.log_scales, self.quats, self.opacity_logits, self.sh)

    @staticmethod
    def from_scene(scene, device="cuda") -> "GaussianTensors":
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(device)
        return GaussianTensors(t(scene.means), t(scene.log_scales), t(scene.quats), t(scene.opacity_logits),
                               t(scene.sh), int(scene.sh_degree))


def default_options(**kw) -> B.ws_options:
    return B.make_options(**kw)


def _aligned_empty(nbytes, device):
    """uint8 device buffer whose start is 256-byte aligned (torch's allocator aligns to 512)."""
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


class Workspace:
    """A growable 256-byte aligned device scratch buffer."""

    def __init__(self, device):
        self.device = device
        self.buf = None

    def get(self, nbytes):
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = _aligned_empty(int(nbytes * 1.25) + 256, self.device)
        return self.buf


def tile_bits(total_tiles: int) -> int:
    return max(1, math.ceil(math.log2(max(total_tiles, 2))))


class Renderer:
    """Render path over a fixed set of cameras (any number of views)."""

    def __init__(self, cams, opts: B.ws_options, device="cuda", capacity=0):
        self.device = torch.device(device)
        self.opts = opts
        self.set_cameras(cams)
        self.capacity = 0
        self.ws_pre = Workspace(self.device)
        self.ws_sort = Workspace(self.device)
        self.ws_render = Workspace(self.device)
        self.ws_bwd = Workspace(self.device)
        self.ws_expand = Workspace(self.device)
        self.tile_vals = None
        self.n = -1
        self.d_num_pairs = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.d_status = torch.zeros(1, dtype=torch.int32, device=self.device)
        self._ensure_capacity(max(int(capacity), 1024))

    # ---------------------------------------------------------- set-up
    def set_cameras(self, cams):
        self.cams = list(cams)
        self.n_views = len(self.cams)
        self.cam_arr = B.camera_array(self.cams)
        self.d_cams = torch.as_tensor(B.camera_bytes(self.cam_arr)).to(self.device)
        self.total_tiles = B.ws_total_tiles(self.cam_arr, self.n_views, self.opts)
        self.total_bins = B.ws_total_bins(self.cam_arr, self.n_views, self.opts)
        self.image_floats = B.ws_total_image_floats(self.cam_arr, self.n_views)
        self.end_bit = 32 + tile_bits(self.total_bins)
        self.tile_ranges = torch.empty(2 * self.total_tiles, dtype=torch.int32, device=self.device)
        self.images = torch.empty(self.image_floats, dtype=torch.float32, device=self.device)
        self.image_offsets = np.concatenate([[0], np.cumsum([3 * c.width * c.height for c in self.cams])])

    def _ensure_n(self, n):
        if n == self.n:
            return
        self.n = n
        v = self.n_views
        # 48-byte ws_splat records, or 32-byte ws_splat_packed ones (WS_FLAG_PACKED)
        words = (B.PACKED_SPLAT_BYTES if self.packed else B.SPLAT_BYTES) // 4
        self.splats = torch.empty((v * max(n, 1), words), dtype=torch.float32, device=self.device)
        self.tiles_touched = torch.empty(v * max(n, 1), dtype=torch.int32, device=self.device)

    def _ensure_capacity(self, cap):
        if cap <= self.capacity:
            return
        cap = int(cap)
        self.capacity = cap
        kt = torch.int32 if self.keys32 else torch.int64
        self.keys_a = torch.empty(cap, dtype=kt, device=self.device)
        self.vals_a = torch.empty(cap, dtype=torch.int32, device=self.device)
        self.keys_b = torch.empty(cap, dtype=kt, device=self.device)
        self.vals_b = torch.empty(cap, dtype=torch.int32, device=self.device)
        if self.binned:
            self.tile_vals = torch.empty(self.per_bin * cap, dtype=torch.int32, device=self.device)

    @property
    def keys32(self) -> bool:
        """Keys are 32-bit tile (bin) ids (WS_FLAG_KEYS32)."""
        return bool(self.opts.flags & B.WS_FLAG_KEYS32)

    @property
    def packed(self) -> bool:
        """Render inputs packed into 32-byte records (WS_FLAG_PACKED; forward only)."""
        return bool(self.opts.flags & B.WS_FLAG_PACKED)

    @property
    def per_bin(self) -> int:
        return max(int(self.opts.bin_x), 1) * max(int(self.opts.bin_y), 1)

    @property
    def binned(self) -> bool:
        return self.per_bin > 1

    @property
    def lists(self) -> torch.Tensor:
        """The per-tile lists that the render and the backward read."""
        return self.tile_vals if self.binned else self.vals_b

    def image(self, v):
        c = self.cams[v]
        o = int(self.image_offsets[v])
        return self.images[o:o + 3 * c.width * c.height].view(3, c.height, c.width)

    # ----------------------------------------------------------- stages
    def preprocess(self, g: GaussianTensors, stream=None):
        self._ensure_n(g.n)
        need = B.ws_preprocess_workspace_size(g.n, self.n_views, self.capacity, self.opts.flags)
        ws = self.ws_pre.get(need)
        B.ws_preprocess(g.struct(), self.cam_arr, self.d_cams, self.n_views, self.opts, self.splats,
                        self.tiles_touched, self.keys_a, self.vals_a, self.capacity, self.d_num_pairs, self.d_status,
                        ws, ws.numel(), stream)

    def sort(self, n_pairs, device_count=False, stream=None, radix_bits=None):
        rb = self.opts.radix_bits if radix_bits is None else radix_bits
        cap = self.capacity if device_count else n_pairs
        begin = self.begin_bit
        d_n = self.d_num_pairs if device_count else None
        if self.keys32:  # the tile bits are the whole key
            need = B.ws_sort32_workspace_size(max(cap, 1), 0, self.end_bit - 32, rb)
            ws = self.ws_sort.get(need)
            B.ws_sort32(self.keys_a, self.vals_a, self.keys_b, self.vals_b, cap, d_n, self.d_status, 0,
                        self.end_bit - 32, rb, ws, ws.numel(), stream)
            return
        need = B.ws_sort_workspace_size(max(cap, 1), begin, self.end_bit, rb)
        ws = self.ws_sort.get(need)
        B.ws_sort(self.keys_a, self.vals_a, self.keys_b, self.vals_b, cap, d_n, self.d_status, begin, self.end_bit,
                  rb, ws, ws.numel(), stream)

    @property
    def begin_bit(self) -> int:
        """Pairs emitted in depth order only need their tile bits sorted (stable)."""
        return 32 if (self.opts.flags & B.WS_FLAG_DEPTH_FIRST) else 0

    def expand(self, cap, stream=None):
        """Tile lists and ranges from the bin-sorted pairs (bins larger than one tile)."""
        need = B.ws_expand_bins_workspace_size(self.cam_arr, self.n_views, self.opts)
        ws = self.ws_expand.get(need)
        B.ws_expand_bins(self.splats, self.n, self.cam_arr, self.d_cams, self.n_views, self.opts, self.keys_b,
                         self.vals_b, cap, self.d_num_pairs, self.d_status, self.tile_vals, self.per_bin * cap,
                         self.tile_ranges, ws, ws.numel(), stream)

    def render(self, cap, stream=None):
        need = B.ws_render_workspace_size(self.cam_arr, self.n_views, self.opts)
        ws = self.ws_render.get(need)
        if self.binned:
            self.expand(cap, stream)
            B.ws_render(self.splats, self.n, self.cam_arr, self.d_cams, self.n_views, self.opts, None, self.tile_vals,
                        self.per_bin * cap, self.d_num_pairs, self.d_status, self.tile_ranges, self.images, ws,
                        ws.numel(), stream)
            return
        B.ws_render(self.splats, self.n, self.cam_arr, self.d_cams, self.n_views, self.opts, self.keys_b, self.vals_b,
                    cap, self.d_num_pairs, self.d_status, self.tile_ranges, self.images, ws, ws.numel(), stream)

    # ------------------------------------------------------- sequences
    def forward(self, g: GaussianTensors, stream=None) -> int:
        """Plain path: returns the pair count M (read back once per frame).

        The device status word is read after the pre-processing (with M) and
        again after the render, so a sort or render that did not complete (an
        expired bounded wait) raises WsError instead of leaving stale images.
        """
        self.preprocess(g, stream)  # resets the status word
        m = int(self.d_num_pairs.item())
        if m > self.capacity:
            self._ensure_capacity(int(m * 1.2) + 1024)
            self.preprocess(g, stream)
        self._check_status()
        self.num_pairs = m
        if m > 0:
            self.sort(m, stream=stream)
        self.render(m, stream)
        self._check_status()
        return m

    def forward_capacity(self, g: GaussianTensors, stream=None):
        """Device-sized path (no host synchronisation); capacity must already cover M."""
        self.preprocess(g, stream)  # resets the status word
        self.sort(self.capacity, device_count=True, stream=stream)
        self.render(self.capacity, stream)

    def backward(self, g: GaussianTensors, dL_dimages: torch.Tensor, grads=None, stream=None, accumulate=False,
                 check=False):
        """Parameter gradients of the last forward for dL/dimages (same layout as self.images).

        Returns a dict of tensors shaped like the parameters; `grads` may supply them.  With `accumulate` the
        library adds the gradients to `grads` (WS_FLAG_ACCUMULATE_GRADS) instead of overwriting them.  If the
        forward's status word is set, the library writes nothing; `check` reads it afterwards (a host
        synchronisation) and raises WsError.
        """
        if grads is None:
            grads = dict(means=torch.empty_like(g.means), log_scales=torch.empty_like(g.log_scales),
                         quats=torch.empty_like(g.quats), opacity_logits=torch.empty_like(g.opacity_logits),
                         sh=torch.empty_like(g.sh))
        need = B.ws_render_backward_workspace_size(g.n, self.n_views)
        ws = self.ws_bwd.get(need)
        gs = B.make_grads(grads["means"], grads["log_scales"], grads["quats"], grads["opacity_logits"], grads["sh"])
        opts = self.opts
        if accumulate:
            opts = B.ws_options.from_buffer_copy(self.opts)
            opts.flags |= B.WS_FLAG_ACCUMULATE_GRADS
        B.ws_render_backward(g.struct(), self.cam_arr, self.d_cams, self.n_views, opts, self.splats,
                             self.tiles_touched, self.lists, self.tile_ranges, self.images, dL_dimages, self.d_status,
                             gs, ws, ws.numel(), stream)
        if check:
            self._check_status()
        return grads

    def backward_l1(self, g: GaussianTensors, targets: torch.Tensor, loss: torch.Tensor, total=0, grads=None,
                    stream=None, accumulate=False, check=False):
        """Parameter gradients of the L1 loss of the last forward's images against `targets` (same layout as
        self.images), and the loss into `loss` (a one-float device tensor): ws_render_backward_l1, which forms
        dL/dimages inside the compositing adjoint.  `total` as in ws_l1_loss (0: this renderer's image
        elements); the other arguments as in backward()."""
        if grads is None:
            grads = dict(means=torch.empty_like(g.means), log_scales=torch.empty_like(g.log_scales),
                         quats=torch.empty_like(g.quats), opacity_logits=torch.empty_like(g.opacity_logits),
                         sh=torch.empty_like(g.sh))
        if targets.numel() != self.image_floats or not targets.is_contiguous():
            raise ValueError("targets must be a contiguous tensor shaped like the images")
        need = B.ws_render_backward_l1_workspace_size(g.n, self.cam_arr, self.n_views, self.opts)
        ws = self.ws_bwd.get(need)
        gs = B.make_grads(grads["means"], grads["log_scales"], grads["quats"], grads["opacity_logits"], grads["sh"])
        opts = self.opts
        if accumulate:
            opts = B.ws_options.from_buffer_copy(self.opts)
            opts.flags |= B.WS_FLAG_ACCUMULATE_GRADS
        B.ws_render_backward_l1(g.struct(), self.cam_arr, self.d_cams, self.n_views, opts, self.splats,
                                self.tiles_touched, self.lists, self.tile_ranges, self.images, targets, total, loss,
                                self.d_status, gs, ws, ws.numel(), stream)
        if check:
            self._check_status()
        return grads

    def _check_status(self):
        st = int(self.d_status.item())
        if st != 0:
            raise B.WsError(st, B.ws_status_string(st))

    def status(self) -> int:
        return int(self.d_status.item())
