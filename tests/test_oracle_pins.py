"""Pins of the fp64 CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a closed
form, a brute-force definition, an invariant, or an independent library
routine.  The paper prints no worked numeric example (its visual comparison
figure is qualitative), so full-scene image values are pinned only through
brute force and invariants.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen
from scenegen import Camera, Scene

PI = math.pi
Y00 = 0.5 / math.sqrt(PI)


def _cam(W, H, f=None, R=np.eye(3), t=(0.0, 0.0, 0.0), C=None):
    f = f if f is not None else scenegen.focal_for_hfov(W)
    R = np.asarray(R, np.float64)
    t = np.asarray(t, np.float64)
    C = -R.T @ t if C is None else np.asarray(C)
    return Camera(W, H, f, f, W / 2.0, H / 2.0, R, t, C)


def _scene(means, log_scales, quats, logits, sh, deg=0):
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.float32))
    return Scene(f(means), f(log_scales), f(quats), f(logits), f(sh), deg)


def _single(mu, log_s, q, logit, dc):
    return _scene(np.reshape(mu, (3, 1)), np.reshape(log_s, (3, 1)), np.reshape(q, (4, 1)), [logit],
                  np.reshape(dc, (3, 1)))


# ----------------------------------------------------------------- P1: sort

def _sort_cases(rng):
    yield "empty", np.zeros(0, np.uint64)
    for n in (1, 63, 64, 65, 1000, 4097):
        yield f"random{n}", rng.integers(0, 2**63, size=n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=n, dtype=np.uint64)
    yield "equal", np.full(777, 12345, np.uint64)
    yield "sorted", np.arange(500, dtype=np.uint64) * np.uint64(3)
    yield "reversed", np.arange(500, dtype=np.uint64)[::-1].copy()
    yield "high32", (rng.integers(0, 50, size=999, dtype=np.uint64) << np.uint64(32))
    yield "bit0", rng.integers(0, 2, size=999, dtype=np.uint64)
    yield "fewdistinct", rng.integers(0, 4, size=3000, dtype=np.uint64) * np.uint64(0x0101010101010101)


@pytest.mark.parametrize("bits", [(0, 64), (0, 32), (32, 64), (3, 17), (0, 1), (63, 64)])
def test_p1_stable_sort_definition(bits):
    rng = np.random.default_rng(11)
    b0, b1 = bits
    mask = np.uint64(((1 << (b1 - b0)) - 1) << b0) if b1 - b0 < 64 else np.uint64(2**64 - 1)
    for name, keys in _sort_cases(rng):
        vals = np.arange(keys.size, dtype=np.uint32)
        sk, sv = oracle.stable_sort(keys, vals, b0, b1)
        # a permutation that moves each value with its key
        assert np.array_equal(np.sort(sv), vals), name
        assert np.array_equal(keys[sv], sk), name
        mk = sk & mask
        assert np.all(mk[1:] >= mk[:-1]), name  # non-decreasing on the key bits
        ties = mk[1:] == mk[:-1]
        assert np.all(sv[1:][ties] > sv[:-1][ties]), name  # equal digits keep input order
        # an independent stable sort (numpy's) agrees
        order = np.argsort(keys & mask, kind="stable")
        assert np.array_equal(order.astype(np.uint32), sv), name


# ------------------------------------------------- P2-P4: closed-form projections

def test_p2_isotropic_closed_form_footprint():
    W = H = 65
    z_cam, s, logit, dc = 2.5, 0.02, 1.2, 0.7
    cam = _cam(W, H, t=(0.0, 0.0, 3.0))
    q = np.array([0.3, -0.5, 0.2, 0.6])  # rotation is irrelevant for an isotropic Gaussian
    sc = _single([0.0, 0.0, z_cam - 3.0], [math.log(s)] * 3, q, logit, [dc, -0.2, 0.1])
    opts = oracle.Options(sh_degree=0)
    p = oracle.preprocess(sc, cam, opts)
    f = cam.fx
    z = np.float64(np.float32(z_cam - 3.0)) + 3.0
    sf = np.float64(np.float32(math.log(s)))
    var = (f * math.exp(sf) / z) ** 2 + 0.3
    assert np.allclose(p["cov2d"][:, 0], [var, 0.0, var], rtol=1e-12, atol=1e-12)
    assert np.allclose(p["conic"][:, 0], [1 / var, 0.0, 1 / var], rtol=1e-12, atol=1e-15)
    assert np.allclose(p["mean2d"][:, 0], [W / 2, H / 2], atol=1e-12)
    sig = 1.0 / (1.0 + math.exp(-np.float64(np.float32(logit))))
    assert abs(p["opacity"][0] - sig) < 1e-15
    r = oracle.render(sc, cam, opts)
    px, py = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    d2 = (px - W / 2) ** 2 + (py - H / 2) ** 2
    alpha = np.minimum(0.99, sig * np.exp(-d2 / (2 * var)))
    inside = d2 <= 2 * var * math.log(255 * sig)
    assert np.array_equal(inside, alpha >= 1 / 255)  # footprint = lattice points inside the disc
    dcs = np.float32([dc, -0.2, 0.1]).astype(np.float64)
    col = np.maximum(0.0, dcs * Y00 + 0.5)
    expect = col[:, None, None] * np.where(inside, alpha, 0.0)[None]
    assert np.max(np.abs(r["rgb"] - expect)) < 1e-13
    assert p["tiles_touched"][0] > 0


def test_p3_off_axis_isotropic():
    W, H = 200, 100
    cam = _cam(W, H, t=(0.0, 0.0, 3.0))
    x, z_w, s = 0.7, 0.5, 0.03
    sc = _single([x, 0.0, z_w], [math.log(s)] * 3, [1, 0, 0, 0], 2.0, [0.1, 0.1, 0.1])
    p = oracle.preprocess(sc, cam, oracle.Options())
    xf, zf = np.float64(np.float32(x)), np.float64(np.float32(z_w)) + 3.0
    sf = math.exp(np.float64(np.float32(math.log(s))))
    f = cam.fx
    k = (f * sf / zf) ** 2
    assert abs(xf / zf) < 1.3 * W / (2 * f)  # inside the clamp
    assert np.allclose(p["cov2d"][:, 0], [k * (1 + (xf / zf) ** 2) + 0.3, 0.0, k + 0.3], rtol=1e-12, atol=1e-14)
    assert np.allclose(p["mean2d"][:, 0], [f * xf / zf + W / 2, H / 2], rtol=1e-14)


def test_p4_anisotropic_facing_and_quarter_turn():
    W = H = 128
    cam = _cam(W, H, t=(0.0, 0.0, 3.0))
    sx, sy, sz = 0.05, 0.01, 0.02
    ls = [math.log(sx), math.log(sy), math.log(sz)]
    f = cam.fx
    lsf = np.exp(np.float32(ls).astype(np.float64))
    a = (f * lsf[0] / 3.0) ** 2 + 0.3
    b = (f * lsf[1] / 3.0) ** 2 + 0.3
    p0 = oracle.preprocess(_single([0, 0, 0], ls, [1, 0, 0, 0], 1.0, [0, 0, 0]), cam, oracle.Options())
    assert np.allclose(p0["cov2d"][:, 0], [a, 0.0, b], rtol=1e-12, atol=1e-12)
    c45 = math.cos(math.pi / 4)
    p1 = oracle.preprocess(_single([0, 0, 0], ls, [c45, 0, 0, c45], 1.0, [0, 0, 0]), cam, oracle.Options())
    assert np.allclose(p1["cov2d"][:, 0], [b, 0.0, a], rtol=1e-6, atol=1e-6)  # fp32 rounding of cos 45
    # an unnormalised quaternion is normalised inside
    p2 = oracle.preprocess(_single([0, 0, 0], ls, [3.0, 0, 0, 0], 1.0, [0, 0, 0]), cam, oracle.Options())
    assert np.allclose(p2["cov2d"][:, 0], p0["cov2d"][:, 0], rtol=1e-14)


# ------------------------------------------------------ P5: compositing order

def test_p5_two_gaussians_front_to_back():
    W = H = 33
    cam = _cam(W, H, t=(0.0, 0.0, 3.0))
    opts = oracle.Options()
    s = math.log(0.05)
    l1, l2 = 0.4, -0.3
    dc1, dc2 = np.array([0.8, 0.1, -0.5]), np.array([-0.4, 0.9, 0.3])

    def two(z1, z2):
        return _scene([[0, 0], [0, 0], [z1, z2]], [[s, s]] * 3, [[1, 1], [0, 0], [0, 0], [0, 0]], [l1, l2],
                      np.stack([dc1, dc2], axis=1))

    sig = lambda l: 1 / (1 + math.exp(-np.float64(np.float32(l))))
    c1 = np.maximum(0, np.float32(dc1).astype(np.float64) * Y00 + 0.5)
    c2 = np.maximum(0, np.float32(dc2).astype(np.float64) * Y00 + 0.5)
    a1, a2 = min(0.99, sig(l1)), min(0.99, sig(l2))
    r = oracle.render(two(0.0, 0.5), cam, opts)
    centre = r["rgb"][:, H // 2, W // 2]
    assert np.allclose(centre, c1 * a1 + c2 * a2 * (1 - a1), rtol=1e-13)
    r = oracle.render(two(0.5, 0.0), cam, opts)
    centre = r["rgb"][:, H // 2, W // 2]
    assert np.allclose(centre, c2 * a2 + c1 * a1 * (1 - a2), rtol=1e-13)
    # equal depths: ties keep Gaussian-id order
    r = oracle.render(two(0.25, 0.25), cam, opts)
    assert np.allclose(r["rgb"][:, H // 2, W // 2], c1 * a1 + c2 * a2 * (1 - a1), rtol=1e-13)


# ----------------------------------------------- P6: brute force == tiled pipeline

def _tiny_scene(seed, n=300, spread=1.0, deg=0):
    sc = scenegen.random_scene(n, seed, mean_lo=-spread, mean_hi=spread, log_scale_mu=-2.8, log_scale_sd=0.6,
                               logit_sd=2.5, sh_degree=deg, dc_sd=0.5, rest_sd=0.2)
    return sc


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 8), (32, 16)])
@pytest.mark.parametrize("seed", [1, 2])
def test_p6_brute_equals_tiled_tiny(tile, seed):
    sc = _tiny_scene(seed, deg=2)
    cam = scenegen.look_at([0.3, -0.2, -3.0], [0, 0, 0], 72, 40)
    opts = oracle.Options(tile_w=tile[0], tile_h=tile[1], sh_degree=2)
    r = oracle.render(sc, cam, opts)
    b = oracle.render(sc, cam, opts, mode="brute")
    flagged = (np.minimum(r["alpha_margin"], b["alpha_margin"]) < 1e-9)
    assert flagged.mean() < 0.01
    assert np.array_equal(r["rgb"][:, ~flagged], b["rgb"][:, ~flagged])
    assert np.array_equal(r["T"][~flagged], b["T"][~flagged])


def test_p6_brute_equals_tiled_near_plane():
    # camera inside the cloud: Gaussians behind, straddling and just beyond the near plane
    sc = _tiny_scene(7, n=400, spread=1.5, deg=1)
    cam = scenegen.look_at([0.0, 0.0, -0.5], [0, 0, 1], 64, 64)
    opts = oracle.Options(sh_degree=1)
    r = oracle.render(sc, cam, opts)
    b = oracle.render(sc, cam, opts, mode="brute")
    st = r["proj"]["status"]
    assert (st == oracle.STATUS["near"]).sum() > 50 and (st == oracle.STATUS["visible"]).sum() > 50
    flagged = np.minimum(r["alpha_margin"], b["alpha_margin"]) < 1e-9
    assert np.array_equal(r["rgb"][:, ~flagged], b["rgb"][:, ~flagged])


@pytest.mark.slow
def test_p6_brute_equals_tiled_c1_sampled():
    sc, cam = scenegen.c1()
    opts = oracle.Options(sh_degree=0)
    r = oracle.render(sc, cam, opts)
    # brute force over every Gaussian, on a band of two tile rows plus a sparse pixel sample
    mask = np.zeros((cam.height, cam.width), np.uint8)
    mask[96:128] = 1
    mask[::7, ::5] = 1
    b = oracle.render(sc, cam, opts, mode="brute", mask=mask)
    sel = mask.astype(bool) & (np.minimum(r["alpha_margin"], b["alpha_margin"]) >= 1e-9)
    assert sel.sum() > 0.99 * mask.sum()
    assert np.array_equal(r["rgb"][:, sel], b["rgb"][:, sel])


# -------------------------------------------------------- P7: culling invariants

def _alpha_all(proj, W, H):
    u, v = proj["mean2d"]
    A, B, Cc = proj["conic"]
    px, py = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    dx = u[:, None, None] - px[None]
    dy = v[:, None, None] - py[None]
    power = -0.5 * (A[:, None, None] * dx * dx + Cc[:, None, None] * dy * dy) - B[:, None, None] * dx * dy
    return proj["opacity"][:, None, None] * np.exp(power)


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_p7_cull_invariants(seed):
    sc = _tiny_scene(seed, n=250, spread=1.6)
    sc.opacity_logits[:40] = np.float32(-6.0)  # below 1/255
    sc.opacity_logits[40:50] = np.float32(-5.537)  # at the 1/255 boundary
    W, H = 48, 40
    cam = scenegen.look_at([0.2, 0.1, -3.0], [0, 0, 0], W, H)
    opts = oracle.Options(tile_w=8, tile_h=8)
    p = oracle.preprocess(sc, cam, opts)
    st = p["status"]
    ok = (st != oracle.STATUS["near"]) & (st != oracle.STATUS["degenerate"])
    alpha = _alpha_all({k: (v[..., ok] if v.ndim > 1 else v[ok]) for k, v in p.items()}, W, H)
    st_ok = st[ok]
    # (i) culled Gaussians never reach alpha_min at any pixel centre
    culled = st_ok != oracle.STATUS["visible"]
    assert culled.sum() > 40
    assert np.all(alpha[culled] < 1 / 255)
    # (ii) every (pixel, Gaussian) with alpha >= alpha_min lies inside an emitted tile
    keys, vals = oracle.emit(sc, cam, opts)
    tx_n, _ = oracle.tiles_xy(cam, opts)
    emitted = set(zip(vals.tolist(), (keys >> np.uint64(32)).astype(np.int64).tolist()))
    idx = np.nonzero(ok)[0]
    g, yy, xx = np.nonzero(alpha >= 1 / 255)
    for gi, y, x in zip(idx[g], yy, xx):
        assert (int(gi), int((y // 8) * tx_n + x // 8)) in emitted
    # (iii) no splat with sigma < 1/255 is emitted
    low = p["opacity"] < 1 / 255
    assert low.sum() >= 40
    assert not np.any(np.isin(vals, np.nonzero(low)[0]))
    # emission count equals the sum of tiles_touched
    assert keys.size == p["tiles_touched"].sum()


# ------------------------------------------------------ P8: transmittance

def test_p8_transmittance_telescoping():
    sc = _tiny_scene(9, n=600, spread=0.8)
    sc.sh[:] = np.float32(0.5 / Y00)  # every colour channel exactly 1
    W = H = 48
    cam = scenegen.look_at([0.0, 0.0, -2.5], [0, 0, 0], W, H)
    opts = oracle.Options()
    r = oracle.render(sc, cam, opts)
    T = r["T"]
    c = r["proj"]["rgb"][0, 0]
    assert abs(c - 1.0) < 1e-6 and np.all(r["proj"]["rgb"] == c)  # one colour for every splat
    assert np.all(T >= 1e-4) and np.all(T <= 1.0)
    assert (T < 0.01).mean() > 0.05  # some pixels reach the early-termination regime
    for ch in range(3):
        assert np.max(np.abs(r["rgb"][ch] - c * (1.0 - T))) < 1e-12
    # a background shows through with weight T
    opts_bg = oracle.Options(bg=(0.25, 0.5, 1.0))
    rb = oracle.render(sc, cam, opts_bg)
    for ch, bgc in enumerate((0.25, 0.5, 1.0)):
        assert np.max(np.abs(rb["rgb"][ch] - (c * (1.0 - T) + bgc * T))) < 1e-12


# ------------------------------------------------------ P9: spherical harmonics

def test_p9_sh_orthonormal_quadrature():
    xg, wg = np.polynomial.legendre.leggauss(24)  # cos(theta), exact for these polynomials
    nphi = 48
    phi = 2 * np.pi * np.arange(nphi) / nphi
    G = np.zeros((16, 16))
    for ct, w in zip(xg, wg):
        st = math.sqrt(1 - ct * ct)
        for ph in phi:
            Y = oracle.sh_basis([st * math.cos(ph), st * math.sin(ph), ct], 3)
            G += w * (2 * np.pi / nphi) * np.outer(Y, Y)
    assert np.max(np.abs(G - np.eye(16))) < 1e-12


def test_p9_sh_values_and_sign_convention():
    Y = oracle.sh_basis([0.0, 0.0, 1.0], 3)
    assert abs(Y[0] - 1 / (2 * math.sqrt(PI))) < 1e-15
    assert abs(Y[2] - math.sqrt(3 / (4 * PI))) < 1e-15  # Y_10 at the pole
    Y = oracle.sh_basis([1.0, 0.0, 0.0], 3)
    assert abs(Y[3] + math.sqrt(3 / (4 * PI))) < 1e-15  # Condon-Shortley: Y_11(x-axis) < 0
    Y = oracle.sh_basis([0.0, 1.0, 0.0], 3)
    assert abs(Y[1] + math.sqrt(3 / (4 * PI))) < 1e-15
    # addition theorem: sum_m Y_lm(d)^2 = (2l+1)/(4 pi) for every direction
    rng = np.random.default_rng(0)
    for _ in range(20):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        Y = oracle.sh_basis(d, 3)
        for l in range(4):
            assert abs(np.sum(Y[l * l:(l + 1) ** 2] ** 2) - (2 * l + 1) / (4 * PI)) < 1e-13


def test_p9_degree0_view_independent():
    sc = _tiny_scene(12, n=50, spread=0.5, deg=0)
    opts = oracle.Options()
    a = oracle.preprocess(sc, scenegen.look_at([0, 0, -3], [0, 0, 0], 64, 64), opts)
    b = oracle.preprocess(sc, scenegen.look_at([2.5, -1.0, -1.0], [0, 0, 0], 64, 64), opts)
    assert np.array_equal(a["rgb"], b["rgb"])


# --------------------------------------------------------------- P10: quaternion

def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_p10_quaternion_rotation():
    rng = np.random.default_rng(2)
    for _ in range(50):
        q = rng.standard_normal(4) * rng.uniform(0.1, 5.0)
        R = oracle.quat_to_rotmat(q)
        assert np.max(np.abs(R @ R.T - np.eye(3))) < 1e-14
        assert abs(np.linalg.det(R) - 1.0) < 1e-14
        qh = q / np.linalg.norm(q)
        v = rng.standard_normal(3)
        rv = _qmul(_qmul(qh, np.concatenate([[0.0], v])), qh * np.array([1, -1, -1, -1]))[1:]
        assert np.allclose(R @ v, rv, atol=1e-13)


def test_p10_covariance_eigenvalues_via_projection():
    # an isotropic pair of axes facing the camera: projected covariance eigenvalues equal
    # (f s_k / z)^2 + 0.3 for the two in-plane axes whatever the in-plane rotation
    W = H = 128
    cam = _cam(W, H, t=(0.0, 0.0, 3.0))
    rng = np.random.default_rng(8)
    ls = [math.log(0.04), math.log(0.01), math.log(0.02)]
    lsf = np.exp(np.float32(ls).astype(np.float64))
    f = cam.fx
    want = np.sort([(f * lsf[0] / 3) ** 2 + 0.3, (f * lsf[1] / 3) ** 2 + 0.3])
    for _ in range(10):
        th = rng.uniform(0, 2 * np.pi)
        q = [math.cos(th / 2), 0, 0, math.sin(th / 2)]  # rotation about the optical axis
        p = oracle.preprocess(_single([0, 0, 0], ls, q, 1.0, [0, 0, 0]), cam, oracle.Options())
        a, b, c = p["cov2d"][:, 0]
        ev = np.sort(np.linalg.eigvalsh([[a, b], [b, c]]))
        assert np.allclose(ev, want, rtol=1e-6)


# -------------------------------------------------- P12/P13: gradients of the oracle

def _param_vec(sc):
    return [("means", sc.means), ("log_scales", sc.log_scales), ("quats", sc.quats),
            ("opacity_logits", sc.opacity_logits), ("sh", sc.sh)]


class _Scene64:
    """fp64 parameters (finite differences need perturbations below fp32 resolution)."""

    def __init__(self, sc):
        self.means = sc.means.astype(np.float64)
        self.log_scales = sc.log_scales.astype(np.float64)
        self.quats = sc.quats.astype(np.float64)
        self.opacity_logits = sc.opacity_logits.astype(np.float64)
        self.sh = sc.sh.astype(np.float64)
        self.sh_degree = sc.sh_degree

    @property
    def n(self):
        return self.means.shape[1]


@pytest.mark.slow
def test_p12_finite_differences_fd_scene():
    sc32, cam = scenegen.fd_scene()
    sc = _Scene64(sc32)
    opts = oracle.Options(sh_degree=3)
    rng = np.random.default_rng(123)
    wts = rng.standard_normal((3, cam.height, cam.width))
    res = oracle.forward_backward(sc, cam, opts, wts)
    assert res["image"].max() > 0.05
    grads = res["grads"]
    probes = []
    for name, arr in _param_vec(sc):
        flat_n = arr.size
        picks = rng.choice(flat_n, size=min(flat_n, 120 if name == "sh" else 60), replace=False)
        probes += [(name, int(p)) for p in picks]
    checked = skipped = 0
    worst = 0.0
    gscale = {name: np.sqrt(np.mean(grads[name] ** 2)) for name in grads}
    for name, p in probes:
        arr = getattr(sc, name)
        flat = arr.reshape(-1)
        x0 = flat[p]
        h = 1e-6 * max(1.0, abs(x0))
        flat[p] = x0 + h
        rp = oracle.forward_backward(sc, cam, opts, None)
        flat[p] = x0 - h
        rm = oracle.forward_backward(sc, cam, opts, None)
        flat[p] = x0
        if rp["hash"] != rm["hash"] or rp["hash"] != res["hash"]:
            skipped += 1
            continue
        fd = (np.sum(wts * rp["image"]) - np.sum(wts * rm["image"])) / (2 * h)
        g = grads[name].reshape(-1)[p]
        err = abs(fd - g) / max(abs(g), 1e-3 * gscale[name], 1e-12)
        worst = max(worst, err)
        assert err < 1e-5, (name, p, fd, g)
        checked += 1
    assert checked > 0.9 * len(probes), (checked, skipped)
    assert worst < 1e-5


def test_p13_closed_form_gradients_single_gaussian():
    W = H = 33
    cam = _cam(W, H, t=(0.0, 0.0, 3.0))
    logit, dc = 0.25, [0.625, -0.125, 0.25]  # exact in fp32
    sc = _Scene64(_single([0.0, 0.0, 0.0], [math.log(0.05)] * 3, [1, 0, 0, 0], logit, dc))
    opts = oracle.Options()
    dL = np.zeros((3, H, W))
    dL[0, H // 2, W // 2] = 1.0  # L = red channel of the centre pixel
    res = oracle.forward_backward(sc, cam, opts, dL)
    sig = 1 / (1 + math.exp(-logit))
    alpha = sig  # the centre pixel sits exactly on the projected mean: power = 0
    c_red = dc[0] * Y00 + 0.5
    assert abs(res["grads"]["sh"][0, 0] - Y00 * alpha) < 1e-14
    assert abs(res["grads"]["opacity_logits"][0] - c_red * sig * (1 - sig)) < 1e-14
    # at the centre the power is stationary: no gradient to the mean's screen position
    assert np.all(np.abs(res["splat_grad"][0, :2]) < 1e-14)
    # off-centre pixel: dC/du = c * alpha * dpower/du, dpower/du = -(A dx + B dy)
    dL = np.zeros((3, H, W))
    dL[1, H // 2, W // 2 + 2] = 1.0
    res = oracle.forward_backward(sc, cam, opts, dL)
    A = oracle.preprocess(sc, cam, opts)["conic"][0, 0]
    dx = (W / 2) - (W // 2 + 2 + 0.5)
    a_off = sig * math.exp(-0.5 * A * dx * dx)
    c_green = dc[1] * Y00 + 0.5
    assert abs(res["splat_grad"][0, 0] - c_green * a_off * (-A * dx)) < 1e-12
    assert abs(res["splat_grad"][0, 7] - a_off) < 1e-14


# ------------------------------- pins that involve a rotated camera and scene

def _rot_from_quat(q):
    """Rotation matrix by rotating the basis vectors with quaternion products."""
    q = np.asarray(q, np.float64) / np.linalg.norm(q)
    cols = [_qmul(_qmul(q, np.concatenate([[0.0], e])), q * np.array([1, -1, -1, -1]))[1:] for e in np.eye(3)]
    return np.stack(cols, axis=1)


def test_p3b_projected_covariance_is_first_order_projection():
    """EWA: Sigma' - lowpass I = J Sigma_cam J^T with J the Jacobian of the pinhole map."""
    rng = np.random.default_rng(21)
    from types import SimpleNamespace
    for trial in range(20):
        Rc = _rot_from_quat(rng.standard_normal(4))
        C = rng.uniform(-1, 1, size=3) - Rc[2] * 4.0  # camera 4 units behind the origin
        t = -Rc @ C
        W, H, f = 320, 240, 300.0
        cam = SimpleNamespace(width=W, height=H, fx=f, fy=f * 1.1, cx=W / 2, cy=H / 2, R=Rc, t=t, C=C)
        mu = rng.uniform(-0.5, 0.5, size=3)
        ls = rng.normal(-2.5, 0.7, size=3)
        q = rng.standard_normal(4)
        sc = _Scene64(_single(mu, ls, q, 2.0, [0, 0, 0]))
        sc.means[:, 0], sc.log_scales[:, 0], sc.quats[:, 0] = mu, ls, q
        p = oracle.preprocess(sc, cam, oracle.Options())
        assert p["status"][0] in (0, 4)
        pc = Rc @ mu + t

        def proj(x):
            return np.array([cam.fx * x[0] / x[2] + cam.cx, cam.fy * x[1] / x[2] + cam.cy])

        J = np.stack([(proj(pc + 1e-6 * e) - proj(pc - 1e-6 * e)) / 2e-6 for e in np.eye(3)], axis=1)
        Rq = _rot_from_quat(q)
        Sig = Rq @ np.diag(np.exp(2 * ls)) @ Rq.T
        want = J @ (Rc @ Sig @ Rc.T) @ J.T + 0.3 * np.eye(2)
        got = np.array([[p["cov2d"][0, 0], p["cov2d"][1, 0]], [p["cov2d"][1, 0], p["cov2d"][2, 0]]])
        assert np.allclose(got, want, rtol=1e-6, atol=1e-6 * np.abs(want).max()), trial
        assert np.allclose(p["mean2d"][:, 0], proj(pc), rtol=1e-13)
        assert abs(p["z"][0] - pc[2]) < 1e-12


def test_p9b_sh_view_direction():
    """Colour uses d = (X - C)/|X - C| from the camera centre to the Gaussian."""
    from types import SimpleNamespace
    rng = np.random.default_rng(4)
    for _ in range(10):
        Rc = _rot_from_quat(rng.standard_normal(4))
        C = rng.uniform(-2, 2, size=3)
        cam = SimpleNamespace(width=64, height=64, fx=60.0, fy=60.0, cx=32.0, cy=32.0, R=Rc, t=-Rc @ C, C=C)
        mu = C + Rc[2] * 2.0 + rng.uniform(-0.3, 0.3, size=3)
        k = rng.normal(0, 0.3, size=(3 * 16,))
        sc = _Scene64(_single(mu, [-3, -3, -3], [1, 0, 0, 0], 2.0, [0, 0, 0]))
        sc.sh_degree = 3
        sc.means[:, 0] = mu
        sc.sh = np.ascontiguousarray(k.reshape(48, 1))
        p = oracle.preprocess(sc, cam, oracle.Options(sh_degree=3))
        d = (mu - C) / np.linalg.norm(mu - C)
        x, y, z = d
        # degree <= 1 part written from the textbook real basis with the Condon-Shortley sign
        Y = oracle.sh_basis(d, 3)
        assert abs(Y[1] + math.sqrt(3 / (4 * PI)) * y) < 1e-15
        assert abs(Y[2] - math.sqrt(3 / (4 * PI)) * z) < 1e-15
        assert abs(Y[3] + math.sqrt(3 / (4 * PI)) * x) < 1e-15
        want = np.maximum(0.0, k.reshape(16, 3).T @ Y + 0.5)
        assert np.allclose(p["rgb"][:, 0], want, rtol=1e-13, atol=1e-14)


def test_p10b_world_rotation_invariance():
    """Rotating the scene and the camera together leaves the image unchanged."""
    from types import SimpleNamespace
    sc32 = _tiny_scene(31, n=200, spread=0.7, deg=0)
    sc = _Scene64(sc32)
    W = H = 48
    cam0 = scenegen.look_at([0.4, -0.3, -2.8], [0, 0, 0], W, H)
    R0, t0, C0 = (np.asarray(a, np.float64) for a in (cam0.R, cam0.t, cam0.C))
    opts = oracle.Options()
    base = oracle.forward_backward(sc, SimpleNamespace(width=W, height=H, fx=cam0.fx, fy=cam0.fy, cx=cam0.cx,
                                                       cy=cam0.cy, R=R0, t=t0, C=C0), opts)["image"]
    rng = np.random.default_rng(5)
    for _ in range(3):
        qQ = rng.standard_normal(4)
        qQ /= np.linalg.norm(qQ)
        Q = _rot_from_quat(qQ)
        rot = _Scene64(sc32)
        rot.means = np.ascontiguousarray(Q @ sc.means)
        rot.quats = np.ascontiguousarray(np.stack([_qmul(qQ, sc.quats[:, i]) for i in range(sc.n)], axis=1))
        cam = SimpleNamespace(width=W, height=H, fx=cam0.fx, fy=cam0.fy, cx=cam0.cx, cy=cam0.cy, R=R0 @ Q.T,
                              t=t0, C=Q @ C0)
        img = oracle.forward_backward(rot, cam, opts)["image"]
        assert np.max(np.abs(img - base)) < 1e-9


def test_p3c_single_anisotropic_image_from_numeric_covariance():
    """One rotated anisotropic Gaussian: every pixel equals c * alpha with alpha from inv(Sigma')."""
    from types import SimpleNamespace
    rng = np.random.default_rng(77)
    for trial in range(8):
        Rc = _rot_from_quat(rng.standard_normal(4))
        C = -Rc[2] * 3.0
        W, H, f = 96, 80, 120.0
        cam = SimpleNamespace(width=W, height=H, fx=f, fy=f, cx=W / 2, cy=H / 2, R=Rc, t=-Rc @ C, C=C)
        mu = rng.uniform(-0.2, 0.2, size=3)
        ls = np.array([-1.6, -3.0, -2.5]) + rng.normal(0, 0.2, size=3)
        q = rng.standard_normal(4)
        sc = _Scene64(_single(mu, ls, q, 1.5, [0.4, 0.2, -0.1]))
        sc.means[:, 0], sc.log_scales[:, 0], sc.quats[:, 0] = mu, ls, q
        opts = oracle.Options()
        p = oracle.preprocess(sc, cam, opts)
        cov = np.array([[p["cov2d"][0, 0], p["cov2d"][1, 0]], [p["cov2d"][1, 0], p["cov2d"][2, 0]]])
        conic = np.linalg.inv(cov)
        assert np.allclose(p["conic"][:, 0], [conic[0, 0], conic[0, 1], conic[1, 1]], rtol=1e-12)
        pc = Rc @ mu + cam.t
        proj = lambda x: np.array([f * x[0] / x[2] + W / 2, f * x[1] / x[2] + H / 2])
        J = np.stack([(proj(pc + 1e-6 * e) - proj(pc - 1e-6 * e)) / 2e-6 for e in np.eye(3)], axis=1)
        Rq = _rot_from_quat(q)
        cov_num = J @ (Rc @ Rq @ np.diag(np.exp(2 * ls)) @ Rq.T @ Rc.T) @ J.T + 0.3 * np.eye(2)
        assert abs(cov_num[0, 1]) > 1e-2 * math.sqrt(cov_num[0, 0] * cov_num[1, 1])  # really anisotropic and tilted
        Q = np.linalg.inv(cov_num)
        m = proj(pc)
        img = oracle.forward_backward(sc, cam, opts)["image"]
        sig = 1 / (1 + math.exp(-sc.opacity_logits[0]))
        col = p["rgb"][:, 0]
        px, py = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
        d = np.stack([px - m[0], py - m[1]], axis=-1)
        q2 = np.einsum("...i,ij,...j->...", d, Q, d)
        alpha = np.minimum(0.99, sig * np.exp(-0.5 * q2))
        safe = np.abs(np.log(255 * alpha)) > 1e-4  # away from the skip threshold (FD Jacobian error)
        expect = np.where(alpha >= 1 / 255, alpha, 0.0)
        assert np.allclose(img[:, safe], col[:, None] * expect[safe][None], rtol=1e-5, atol=1e-7), trial


def test_p17_non_finite_colour_culls_as_degenerate():
    """A non-finite SH coefficient makes the colour non-finite: the splat is culled as degenerate
    (reading of the non-finite-input rule) and contributes nowhere, in either compositing mode."""
    mu = np.array([[0.0, 0.05], [0.0, 0.0], [3.0, 3.2]])
    sc = _scene(mu, np.full((3, 2), -2.5), np.tile([[1.0], [0.0], [0.0], [0.0]], (1, 2)), [2.0, 2.0],
                np.array([[0.4, np.nan], [0.1, 0.2], [0.3, np.inf]]))
    cam = _cam(48, 40)
    opts = oracle.Options()
    pre = oracle.preprocess(sc, cam, opts)
    assert list(pre["status"]) == [oracle.STATUS["visible"], oracle.STATUS["degenerate"]]
    alone = _single(mu[:, 0], [-2.5] * 3, [1.0, 0, 0, 0], 2.0, [0.4, 0.1, 0.3])
    for mode in ("tiled", "brute"):
        img = oracle.render(sc, cam, opts, mode=mode)["rgb"]
        ref = oracle.render(alone, cam, opts, mode=mode)["rgb"]
        assert np.all(np.isfinite(img)) and np.array_equal(img, ref), mode


def _real_sh_from_complex(l, m, d):
    """Real SH of reading A10 built from scipy's complex Y_l^|m| (which carries the Condon-Shortley phase):
    sqrt(2) Re for m > 0, sqrt(2) Im for m < 0, Y_l^0 for m = 0.  Independent of the oracle's polynomials."""
    from scipy.special import sph_harm_y
    theta = math.acos(max(-1.0, min(1.0, d[2])))
    phi = math.atan2(d[1], d[0])
    c = complex(sph_harm_y(l, abs(m), theta, phi))
    if m == 0:
        return c.real
    return math.sqrt(2.0) * (c.real if m > 0 else c.imag)


def test_p9c_sh_every_term_against_scipy():
    """Every basis function Y_k, k = l^2 + l + m (degrees 0-3), value and sign, equals the real SH built from
    scipy's complex spherical harmonics under reading A10.  A sign flip, a swap of two functions of one degree,
    a wrong constant or a wrong index fails here (orthonormality alone is blind to the first two)."""
    rng = np.random.default_rng(2602)
    dirs = [np.array(v, float) for v in ([1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [0, -1, 0], [0, 0, -1])]
    for _ in range(200):
        v = rng.standard_normal(3)
        dirs.append(v / np.linalg.norm(v))
    worst = 0.0
    for d in dirs:
        Y = oracle.sh_basis(d, 3)
        for l in range(4):
            for m in range(-l, l + 1):
                want = _real_sh_from_complex(l, m, d)
                worst = max(worst, abs(Y[l * l + l + m] - want))
    assert worst < 1e-13, worst
    # the basis at a lower degree is the prefix of the degree-3 basis
    for deg in range(3):
        assert np.array_equal(oracle.sh_basis(dirs[7], deg), oracle.sh_basis(dirs[7], 3)[: (deg + 1) ** 2])


def test_p9d_sh_terms_at_chosen_directions():
    """Hand-derived values of degree 2-3 terms (sign and index) where only one or two terms are nonzero."""
    s = 1.0 / math.sqrt(2.0)
    # d = (1, 1, 0)/sqrt 2: xy = 1/2, z = 0
    Y = oracle.sh_basis(np.array([s, s, 0.0]), 3)
    assert abs(Y[4] - 0.5 * math.sqrt(15 / PI) * 0.5) < 1e-15          # m = -2: xy term, positive
    assert abs(Y[5]) < 1e-15 and abs(Y[7]) < 1e-15 and abs(Y[14]) < 1e-15 and abs(Y[10]) < 1e-15
    assert abs(Y[8]) < 1e-15                                             # x^2 - y^2 = 0
    # d = (1, 0, 1)/sqrt 2: xz = 1/2, y = 0
    Y = oracle.sh_basis(np.array([s, 0.0, s]), 3)
    assert abs(Y[7] + 0.5 * math.sqrt(15 / PI) * 0.5) < 1e-15          # m = +1 carries the Condon-Shortley minus
    assert abs(Y[5]) < 1e-15 and abs(Y[4]) < 1e-15 and abs(Y[9]) < 1e-15 and abs(Y[11]) < 1e-15
    # d = +x: the m = +3 cubic is -k3a x (x^2 - 3y^2) = -k3a; m = +1 cubic is -k3c x (4z^2 - x^2 - y^2) = +k3c
    Y = oracle.sh_basis(np.array([1.0, 0.0, 0.0]), 3)
    assert abs(Y[15] + 0.25 * math.sqrt(35 / (2 * PI))) < 1e-15
    assert abs(Y[13] - 0.25 * math.sqrt(21 / (2 * PI))) < 1e-15
    assert abs(Y[8] - 0.25 * math.sqrt(15 / PI)) < 1e-15               # m = +2: x^2 - y^2 = 1
    # d = +y: the m = -3 cubic is -k3a y (3x^2 - y^2) = +k3a
    Y = oracle.sh_basis(np.array([0.0, 1.0, 0.0]), 3)
    assert abs(Y[9] - 0.25 * math.sqrt(35 / (2 * PI))) < 1e-15
    # d = +z: only the m = 0 terms survive, each sqrt((2l+1)/4pi)
    Y = oracle.sh_basis(np.array([0.0, 0.0, 1.0]), 3)
    for l in range(4):
        for m in range(-l, l + 1):
            want = math.sqrt((2 * l + 1) / (4 * PI)) if m == 0 else 0.0
            assert abs(Y[l * l + l + m] - want) < 1e-15, (l, m)


def test_p18_l1_loss_hand_computed():
    """L1 of reading A19 on a hand-computed batch: the mean over every element of every view, sign(0) = 0."""
    img = np.array([1.0, 2.0, 3.0, 4.0])
    tgt = np.array([1.0, 0.0, 5.0, 4.5])
    loss, g = oracle.l1_loss_grad(img, tgt)
    assert loss == (0 + 2 + 2 + 0.5) / 4
    assert np.array_equal(g, [0.0, 0.25, -0.25, -0.25])
    # two views of different sizes: one mean over all 6 elements, not a mean of per-view means
    v0, t0 = np.array([[0.5, 0.5]]), np.array([[0.25, 0.5]])
    v1, t1 = np.array([1.0, 1.0, 1.0, 2.0]), np.array([0.0, 3.0, 1.0, 2.0])
    loss, (g0, g1) = oracle.l1_loss_grad([v0, v1], [t0, t1])
    assert loss == (0.25 + 0 + 1 + 2 + 0 + 0) / 6
    assert g0.shape == (1, 2) and np.array_equal(g0, [[1 / 6, 0.0]])
    assert np.array_equal(g1, [1 / 6, -1 / 6, 0.0, 0.0])
    # the gradient is the subgradient: finite differences away from the kinks
    rng = np.random.default_rng(9)
    a, b = rng.normal(size=50), rng.normal(size=50)
    _, ga = oracle.l1_loss_grad(a, b)
    for i in range(0, 50, 7):
        e = np.zeros(50)
        e[i] = 1e-7
        fd = (oracle.l1_loss_grad(a + e, b)[0] - oracle.l1_loss_grad(a - e, b)[0]) / 2e-7
        assert abs(fd - ga[i]) < 1e-9


def test_p19_packed_ellipse_axes_and_bytes():
    """Sec. 3.2's packing as the oracle models it: the axes of [[a, b], [b, c]] rebuild it exactly, are orthogonal
    and ordered; hand-computed axes of two ellipses; the byte quantisation of colour and opacity."""
    rng = np.random.default_rng(19)
    n = 500
    s1 = np.exp(rng.uniform(-1, 5, n))
    s2 = s1 * np.exp(-rng.uniform(0, 5, n))
    th = rng.uniform(0, np.pi, n)
    c_, s_ = np.cos(th), np.sin(th)
    a = c_ * c_ * s1 * s1 + s_ * s_ * s2 * s2
    c = s_ * s_ * s1 * s1 + c_ * c_ * s2 * s2
    b = c_ * s_ * (s1 * s1 - s2 * s2)
    ax = oracle.ellipse_axes(np.stack([a, b, c]))
    a1, a2 = ax[:2], ax[2:]
    rebuilt = np.stack([a1[0] ** 2 + a2[0] ** 2, a1[0] * a1[1] + a2[0] * a2[1], a1[1] ** 2 + a2[1] ** 2])
    assert np.allclose(rebuilt, np.stack([a, b, c]), rtol=1e-10, atol=1e-10 * s1 * s1)
    assert np.all(np.abs((a1 * a2).sum(0)) <= 1e-10 * s1 * s1)
    n1, n2 = np.hypot(*a1), np.hypot(*a2)
    assert np.allclose(n1, s1, rtol=1e-9) and np.allclose(n2, s2, rtol=1e-6)
    # diag(4, 1): axes (2, 0) and (0, 1); [[2, 1], [1, 2]]: l1 = 3 along (1, 1)/sqrt 2, l2 = 1 along (-1, 1)/sqrt 2
    got = oracle.ellipse_axes(np.array([[4.0, 2.0], [0.0, 1.0], [1.0, 2.0]]))
    r = math.sqrt(0.5)
    assert np.allclose(got[:, 0], [2, 0, 0, 1]) and np.allclose(got[:, 1], [math.sqrt(3) * r, math.sqrt(3) * r, -r, r])
    # a > c with b < 0 and a < c: the eigenvector equation holds for axis1
    for cov in ([5.0, -2.0, 1.0], [1.0, 0.7, 3.0]):
        A = np.array([[cov[0], cov[1]], [cov[1], cov[2]]])
        g = oracle.ellipse_axes(np.array(cov).reshape(3, 1))[:, 0]
        lam = np.linalg.eigvalsh(A)[1]
        assert np.allclose(A @ g[:2], lam * g[:2], rtol=1e-12)
    # bytes: floor(255 x + 1/2) / 255, colours clamped at 1
    proj = dict(status=np.zeros(4, np.int8), cov2d=np.tile([[2.0], [0.0], [2.0]], (1, 4)), conic=np.zeros((3, 4)),
                opacity=np.array([1 / 255, 0.5, 0.99, 1.0]), rgb=np.array([[0.0, 0.5, 1.3, 0.2 / 255]] * 3))
    conic, op, rgb = oracle.pack_quantise(proj)
    assert np.array_equal(op * 255, [1, 128, 252, 255])
    assert np.array_equal(rgb[0] * 255, [0, 128, 255, 0])
    # the axes (sqrt 2, 0), (0, sqrt 2) in fp16: sqrt 2 rounds to 1.4140625, the conic is its inverse square
    assert np.array_equal(conic[:, 0], [1 / 1.4140625 ** 2, 0.0, 1 / 1.4140625 ** 2])


def test_p20_results_do_not_depend_on_the_thread_count():
    """The oracle's loops over independent Gaussians, tiles and pixel rows give the same bits on 1 and on 4
    host threads: tiled and brute compositing, decision outcomes, emission and gradients."""
    sc = _tiny_scene(77, n=600, spread=1.0, deg=1)
    cam = scenegen.look_at([0.3, -0.2, -2.5], [0, 0, 0], 72, 56)
    opts = oracle.Options(sh_degree=1)
    runs = []
    n0 = oracle.max_threads()
    for k in (1, 4):
        oracle.set_threads(k)
        t = oracle.render(sc, cam, opts, outcomes=True)
        b = oracle.render(sc, cam, opts, mode="brute")
        fb = oracle.forward_backward(sc, cam, opts, np.ones((3, cam.height, cam.width)))
        runs.append((t, b, fb))
    oracle.set_threads(n0)
    (t1, b1, f1), (t4, b4, f4) = runs
    for key in ("rgb", "T", "n_eval", "hash"):
        assert np.array_equal(t1[key], t4[key]) and np.array_equal(b1[key], b4[key]), key
    assert np.array_equal(t1["keys"], t4["keys"]) and np.array_equal(t1["sorted_vals"], t4["sorted_vals"])
    for key in ("pix", "n_out", "rgb", "bound"):
        assert np.array_equal(t1["outcomes"][key], t4["outcomes"][key]), key
    for key in f1["grads"]:
        assert np.array_equal(f1["grads"][key], f4["grads"][key]), key
