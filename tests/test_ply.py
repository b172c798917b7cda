"""The trained-scene PLY reader: round trips of seeded scenes of every SH degree, the channel-major f_rest
layout against a hand-built file, and malformed files rejected with a message."""
import numpy as np
import pytest

import scenegen
from paper_2602_03207_amd.ply import read_ply, write_ply


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_round_trip_is_bit_exact(tmp_path, deg):
    sc = scenegen.random_scene(777, 40 + deg, sh_degree=deg, dc_sd=0.5, rest_sd=0.2)
    p = tmp_path / f"s{deg}.ply"
    write_ply(p, sc)
    g = read_ply(p)
    assert g.sh_degree == deg and g.n == sc.n
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        a, b = getattr(g, k), getattr(sc, k)
        assert a.dtype == np.float32 and a.shape == b.shape and np.array_equal(a.view(np.uint32), b.view(np.uint32)), k


def test_ascii_round_trip(tmp_path):
    sc = scenegen.random_scene(50, 3, sh_degree=1, dc_sd=0.5, rest_sd=0.2)
    p = tmp_path / "a.ply"
    write_ply(p, sc, binary=False)
    g = read_ply(p)
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        assert np.array_equal(getattr(g, k), getattr(sc, k)), k


def test_channel_major_rest_layout(tmp_path):
    """A hand-written degree-1 file: f_rest_0..2 are R's coefficients 1..3, f_rest_3..5 G's, f_rest_6..8 B's;
    extra properties of other types (normals as doubles, a uchar) are skipped."""
    names = ["x", "y", "z", "nx", "f_dc_0", "f_dc_1", "f_dc_2"] + [f"f_rest_{i}" for i in range(9)] + \
        ["opacity", "scale_0", "scale_1", "scale_2", "rot_0", "rot_1", "rot_2", "rot_3", "flag"]
    types = {"nx": "f8", "flag": "u1"}
    dt = np.dtype([(nm, "<" + types.get(nm, "f4")) for nm in names])
    rec = np.zeros(2, dt)
    for i, nm in enumerate(names):
        rec[nm] = [i + 0.5, 100 + i] if nm != "flag" else [1, 2]
    hdr = "ply\nformat binary_little_endian 1.0\ncomment hand-built\nelement vertex 2\n"
    tname = {"f4": "float", "f8": "double", "u1": "uchar"}
    hdr += "".join(f"property {tname[types.get(nm, 'f4')]} {nm}\n" for nm in names) + "end_header\n"
    p = tmp_path / "h.ply"
    p.write_bytes(hdr.encode() + rec.tobytes())
    g = read_ply(p)
    assert g.sh_degree == 1 and g.sh.shape == (12, 2)
    val = lambda nm: rec[nm].astype(np.float32)  # noqa: E731
    for c in range(3):
        assert np.array_equal(g.sh[c], val(f"f_dc_{c}"))
        for k in range(1, 4):
            assert np.array_equal(g.sh[k * 3 + c], val(f"f_rest_{c * 3 + k - 1}")), (c, k)
    assert np.array_equal(g.quats[0], val("rot_0")) and np.array_equal(g.opacity_logits, val("opacity"))


def test_malformed_files_are_rejected(tmp_path):
    sc = scenegen.random_scene(10, 1, sh_degree=0)
    good = tmp_path / "g.ply"
    write_ply(good, sc)
    raw = good.read_bytes()
    bad = tmp_path / "b.ply"
    bad.write_bytes(raw[:-7])
    with pytest.raises(ValueError, match="truncated"):
        read_ply(bad)
    bad.write_bytes(b"plx\n" + raw[4:])
    with pytest.raises(ValueError, match="magic"):
        read_ply(bad)
    bad.write_bytes(raw.replace(b"property float opacity\n", b"property float opacitx\n"))
    with pytest.raises(ValueError, match="lacks"):
        read_ply(bad)
    bad.write_bytes(raw.replace(b"element vertex 10\n", b"element vertex 10\nproperty list uchar int face\n"))
    with pytest.raises(ValueError, match="list"):
        read_ply(bad)


@pytest.mark.gpu
def test_ply_scene_renders_like_the_oracle(tmp_path):
    """A degree-3 scene written to PLY and read back renders on the GPU as the oracle renders the original."""
    import oracle
    from _helpers import assert_image_parity, gpu_options, oracle_options
    from paper_2602_03207_amd.pipeline import GaussianTensors, Renderer
    sc = scenegen.random_scene(3000, 44, mean_lo=-1.2, mean_hi=1.2, log_scale_mu=-3.0, sh_degree=3, dc_sd=0.5,
                               rest_sd=0.3)
    p = tmp_path / "scene.ply"
    write_ply(p, sc)
    g = read_ply(p)
    cam = scenegen.look_at([1.1, -0.6, -2.6], [0, 0, 0], 144, 112)
    r = Renderer([cam], gpu_options(sh_degree=3))
    r.forward(GaussianTensors.from_scene(g))
    ref = oracle.render(sc, cam, oracle_options(sh_degree=3), outcomes=True)
    assert r.num_pairs == ref["keys"].size
    assert_image_parity(r.image(0).cpu().numpy(), ref)
