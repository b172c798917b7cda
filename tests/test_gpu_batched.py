"""Batched forward (one graph replay for many views), the ordered persistent render and the autotuner."""
import json

import numpy as np
import pytest

import scenegen
from _helpers import gpu_options

pytestmark = pytest.mark.gpu


def _views():
    rng = np.random.default_rng(11)
    res = [(128, 128), (160, 90), (96, 120), (200, 64), (64, 64)]
    return scenegen.orbit_cameras(rng, len(res), res)


def test_batched_forward_graph_equals_plain_and_replays_consistently():
    import torch
    from paper_2602_03207_amd import binding as B
    from paper_2602_03207_amd.batched import BatchedForward, PlainForward
    from paper_2602_03207_amd.pipeline import GaussianTensors
    scene = scenegen.random_scene(6000, 12, log_scale_mu=-3.2, sh_degree=3, dc_sd=0.5, rest_sd=0.2)
    g = GaussianTensors.from_scene(scene)
    cams = _views()
    opts = gpu_options(sh_degree=3, flags=B.WS_FLAG_DEPTH_FIRST | B.WS_FLAG_ORDERED_RENDER)
    plain = PlainForward(cams, opts, g)
    plain.step()
    torch.cuda.synchronize()
    want = plain.images().clone()
    bf = BatchedForward(cams, opts, g)
    bf.capture()
    for rep in range(3):
        with torch.cuda.stream(bf.stream):  # eager work between replays; the graph must overwrite it
            bf.r.images.fill_(-1.0)
            bf.r.tile_ranges.fill_(7)
        bf.replay()
        bf.check()
        assert torch.equal(bf.r.images.view(torch.int32), want.view(torch.int32)), rep
    bf.close()


def test_autotune_picks_a_candidate_and_caches_it(tmp_path):
    from paper_2602_03207_amd import binding as B
    from paper_2602_03207_amd.autotune import autotune
    from paper_2602_03207_amd.pipeline import GaussianTensors
    scene, _ = scenegen.c1()
    g = GaussianTensors.from_scene(scene)
    cams = _views()[:3]
    base = gpu_options(flags=B.WS_FLAG_ORDERED_RENDER)
    cache = str(tmp_path / "tune.json")
    tiles, radix, bins = ((16, 16), (8, 8)), (6, 8), ((1, 1), (2, 2))
    # every candidate's images must equal the first's (the tuner raises otherwise), bins included
    res = autotune(g, cams, base, tiles=tiles, radix_bits=radix, reps=2, cache_path=cache, bins=bins)
    assert (res.tile_w, res.tile_h) in tiles and res.radix_bits in radix and not res.cached
    assert (res.bin_x, res.bin_y) in bins
    assert len(res.table) == 8 and res.ms == min(row[6] for row in res.table)
    assert res.ordered == bool(base.flags & B.WS_FLAG_ORDERED_RENDER)  # the options' schedule by default
    stored = json.load(open(cache))
    assert res.signature in stored
    again = autotune(g, cams, base, tiles=tiles, radix_bits=radix, reps=2, cache_path=cache, bins=bins)
    assert again.cached and (again.tile_w, again.tile_h, again.radix_bits, again.bin_x, again.bin_y) == \
        (res.tile_w, res.tile_h, res.radix_bits, res.bin_x, res.bin_y)
    o = res.apply(base)
    assert (o.tile_w, o.tile_h, o.radix_bits, o.bin_x, o.bin_y) == \
        (res.tile_w, res.tile_h, res.radix_bits, res.bin_x, res.bin_y)
    assert o.flags == base.flags
    # a search without bins is cached under another signature
    plain = autotune(g, cams, base, tiles=tiles, radix_bits=radix, reps=2, cache_path=cache)
    assert not plain.cached and (plain.bin_x, plain.bin_y) == (1, 1) and len(plain.table) == 4
    # both render schedules: every candidate's images equal the first's, the choice is applied to the flags
    both = autotune(g, cams, base, tiles=((16, 16),), radix_bits=(8,), reps=2, ordered=(False, True))
    assert len(both.table) == 2 and {row[5] for row in both.table} == {False, True}
    ob = both.apply(base)
    assert bool(ob.flags & B.WS_FLAG_ORDERED_RENDER) == both.ordered
    assert (ob.flags & ~B.WS_FLAG_ORDERED_RENDER) == (base.flags & ~B.WS_FLAG_ORDERED_RENDER)
