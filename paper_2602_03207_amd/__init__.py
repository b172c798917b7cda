"""MI355X-native 3D Gaussian Splatting render path (WebSplatter, arXiv 2602.03207).

The compute lives in libwebsplat.so (hand-written HIP for gfx950, C ABI in
include/websplat.h).  This package is its thin Python side:

* `binding`   ctypes marshalling of the C functions (same names: ws_preprocess,
              ws_sort, ws_render, ws_render_backward, ...);
* `pipeline`  device buffers and call sequences (plain and device-sized);
* `autograd`  torch.autograd.Function over the forward and backward calls;
* `batched`   multi-view training step captured in a HIP graph;
* `autotune`  choice of tile size and radix width by timing.

Importing the package does not load the library; the first call does, and it
raises if the library has not been built.
"""
from .binding import (WsError, ws_graph_begin, ws_graph_destroy, ws_graph_end, ws_graph_launch, ws_l1_loss,  # noqa: F401
                      ws_last_error, ws_preprocess, ws_render, ws_render_backward, ws_sort, ws_status_string,
                      ws_version)

__all__ = ["binding", "pipeline", "WsError", "ws_preprocess", "ws_sort", "ws_render", "ws_render_backward",
           "ws_l1_loss", "ws_graph_begin", "ws_graph_end", "ws_graph_launch", "ws_graph_destroy", "ws_last_error",
           "ws_status_string", "ws_version"]
