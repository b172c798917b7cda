"""Autotuner for the free parameters of the render path: the tile size, the
radix width of the sort and (optionally) the bins of tiles that pair keys
name.

No parameter changes a result: the images are bit-identical for every
tile size (each splat is tested against the pixel rectangle, not the tile),
the sort is the same stable order for every radix width, and a bin's
expanded lists are its tiles' lists.  The tuner
therefore only times the device-sized forward (`Renderer.forward_capacity`,
the sequence the batched graph replays) for each candidate, keeps the
fastest, and checks on the way that every candidate produced exactly the
same images — a mismatch is an error, never a choice.

Results are cached in a JSON file keyed by the workload's signature (device
name, Gaussian count, SH degree, view resolutions and option flags), so a
later run with the same workload skips the search.
"""
from __future__ import annotations

import json
import os
import statistics
from dataclasses import asdict, dataclass, field

import torch

from . import binding as B
from .pipeline import GaussianTensors, Renderer

TILES = ((16, 16), (8, 8), (16, 8), (32, 16))
RADIX_BITS = (4, 5, 6, 7, 8)
BINS = ((1, 1),)  # bins of tiles searched by default: none (pass e.g. ((1, 1), (2, 2), (4, 2)))


@dataclass
class TuneResult:
    tile_w: int
    tile_h: int
    radix_bits: int
    ms: float
    signature: str
    table: list = field(default_factory=list)  # [tile_w, tile_h, radix_bits, bin_x, bin_y, median ms]
    cached: bool = False
    bin_x: int = 1
    bin_y: int = 1

    def apply(self, opts: B.ws_options) -> B.ws_options:
        """A copy of `opts` with the tuned tile size, radix width and bins."""
        o = B.ws_options.from_buffer_copy(opts)
        o.tile_w, o.tile_h, o.radix_bits = self.tile_w, self.tile_h, self.radix_bits
        o.bin_x, o.bin_y = self.bin_x, self.bin_y
        return o


def signature(g: GaussianTensors, cams, opts: B.ws_options, device=None, bins=BINS) -> str:
    dev = torch.cuda.get_device_name(device)
    res = sorted((c.width, c.height) for c in cams)
    counts = {}
    for r in res:
        counts[r] = counts.get(r, 0) + 1
    views = ",".join(f"{w}x{h}*{k}" for (w, h), k in sorted(counts.items()))
    searched = ",".join(f"{bx}x{by}" for bx, by in bins)
    return f"{dev}|n={g.n}|sh={g.sh_degree}|flags={int(opts.flags)}|{views}|bins={searched}"


def _load_cache(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _time_forward(r: Renderer, g: GaussianTensors, reps: int, stream) -> float:
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    for i in range(reps):
        starts[i].record(stream)
        r.forward_capacity(g, stream=stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    return statistics.median(s.elapsed_time(e) for s, e in zip(starts, ends))


def autotune(g: GaussianTensors, cams, opts: B.ws_options, tiles=TILES, radix_bits=RADIX_BITS, reps=5,
             cache_path=None, headroom=1.1, log=None, bins=BINS) -> TuneResult:
    """Times every (tile, radix width, bins) candidate and returns the fastest."""
    sig = signature(g, cams, opts, bins=bins)
    cache = _load_cache(cache_path)
    if sig in cache:
        return TuneResult(**{**cache[sig], "cached": True})
    stream = torch.cuda.current_stream()
    ref_images = None
    table = []
    for (tw, th), (bx, by) in ((t, b) for t in tiles for b in bins):
        o = B.ws_options.from_buffer_copy(opts)
        o.tile_w, o.tile_h = tw, th
        o.bin_x, o.bin_y = bx, by
        r = Renderer(cams, o)
        m = r.forward(g, stream)  # sizes every buffer, reads M once
        r._ensure_capacity(int(m * headroom) + 4096)
        for rb in radix_bits:
            r.opts.radix_bits = rb
            r.forward_capacity(g, stream=stream)  # warm-up of this radix width
            ms = _time_forward(r, g, reps, stream)
            if r.status() != 0:
                raise B.WsError(r.status(), B.ws_status_string(r.status()))
            if ref_images is None:
                ref_images = r.images.clone()
            elif not torch.equal(r.images.view(torch.int32), ref_images.view(torch.int32)):
                raise RuntimeError(f"images differ for tile {tw}x{th}, radix {rb}, bins {bx}x{by}: "
                                   "tile size, radix width and bins must not change any pixel")
            table.append([tw, th, rb, bx, by, round(ms, 5)])
            if log:
                log(f"autotune: tile {tw}x{th} radix {rb} bins {bx}x{by}: {ms:.4f} ms")
        del r
    best = min(table, key=lambda row: row[5])
    res = TuneResult(tile_w=best[0], tile_h=best[1], radix_bits=best[2], ms=best[5], signature=sig, table=table,
                     bin_x=best[3], bin_y=best[4])
    if cache_path:
        cache = _load_cache(cache_path)
        d = asdict(res)
        d.pop("cached")
        cache[sig] = d
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return res
