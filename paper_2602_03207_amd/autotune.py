"""Autotuner for the free parameters of the render path: the tile size, the
radix width of the sort and (optionally) the bins of tiles that pair keys
name and the render's schedule (one workgroup per tile, or persistent
workgroups taking tiles longest first from a queue).

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
RADIX_BITS = (5, 6, 7, 8, 9, 10)
BINS = ((1, 1),)  # bins of tiles searched by default: none (pass e.g. ((1, 1), (2, 2), (4, 2)))
ORDERED = (None,)  # render schedules searched by default: the one in the options (pass (False, True) for both)


@dataclass
class TuneResult:
    tile_w: int
    tile_h: int
    radix_bits: int
    ms: float
    signature: str
    table: list = field(default_factory=list)  # [tile_w, tile_h, radix_bits, bin_x, bin_y, ordered, median ms]
    cached: bool = False
    bin_x: int = 1
    bin_y: int = 1
    ordered: bool = False

    def apply(self, opts: B.ws_options) -> B.ws_options:
        """A copy of `opts` with the tuned tile size, radix width and bins."""
        o = B.ws_options.from_buffer_copy(opts)
        o.tile_w, o.tile_h, o.radix_bits = self.tile_w, self.tile_h, self.radix_bits
        o.bin_x, o.bin_y = self.bin_x, self.bin_y
        o.flags = _with_ordered(o.flags, self.ordered)
        return o


def _with_ordered(flags: int, ordered) -> int:
    if ordered is None:
        return flags
    return (flags | B.WS_FLAG_ORDERED_RENDER) if ordered else (flags & ~B.WS_FLAG_ORDERED_RENDER)


def signature(g: GaussianTensors, cams, opts: B.ws_options, device=None, bins=BINS, ordered=ORDERED) -> str:
    dev = torch.cuda.get_device_name(device)
    res = sorted((c.width, c.height) for c in cams)
    counts = {}
    for r in res:
        counts[r] = counts.get(r, 0) + 1
    views = ",".join(f"{w}x{h}*{k}" for (w, h), k in sorted(counts.items()))
    searched = ",".join(f"{bx}x{by}" for bx, by in bins)
    sched = ",".join("opts" if o is None else str(int(o)) for o in ordered)
    return f"{dev}|n={g.n}|sh={g.sh_degree}|flags={int(opts.flags)}|{views}|bins={searched}|ordered={sched}"


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
             cache_path=None, headroom=1.1, log=None, bins=BINS, ordered=ORDERED) -> TuneResult:
    """Times every (tile, radix width, bins, render schedule) candidate and returns the fastest."""
    sig = signature(g, cams, opts, bins=bins, ordered=ordered)
    cache = _load_cache(cache_path)
    if sig in cache:
        return TuneResult(**{**cache[sig], "cached": True})
    stream = torch.cuda.current_stream()
    ref_images = None
    table = []
    for (tw, th), (bx, by), od in ((t, b, s) for t in tiles for b in bins for s in ordered):
        o = B.ws_options.from_buffer_copy(opts)
        o.tile_w, o.tile_h = tw, th
        o.bin_x, o.bin_y = bx, by
        o.flags = _with_ordered(o.flags, od)
        odf = bool(o.flags & B.WS_FLAG_ORDERED_RENDER)
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
                raise RuntimeError(f"images differ for tile {tw}x{th}, radix {rb}, bins {bx}x{by}, ordered {odf}: "
                                   "tile size, radix width, bins and render schedule must not change any pixel")
            table.append([tw, th, rb, bx, by, odf, round(ms, 5)])
            if log:
                log(f"autotune: tile {tw}x{th} radix {rb} bins {bx}x{by} ordered {odf}: {ms:.4f} ms")
        del r
    best = min(table, key=lambda row: row[6])
    res = TuneResult(tile_w=best[0], tile_h=best[1], radix_bits=best[2], ms=best[6], signature=sig, table=table,
                     bin_x=best[3], bin_y=best[4], ordered=best[5])
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
