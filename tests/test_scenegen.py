"""Seeded generators: determinism and the shapes of the five workloads."""
import json
import os

import numpy as np
import pytest

import scenegen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _hash(scene):
    return scenegen.sha256_arrays([scene.means, scene.log_scales, scene.quats, scene.opacity_logits, scene.sh])


def test_generators_are_deterministic():
    with open(os.path.join(GOLDEN, "scenegen_sha256.json")) as f:
        want = json.load(f)
    s1, cam1 = scenegen.c1()
    assert _hash(s1) == want["C1"]
    s2, cam2 = scenegen.c2()
    assert _hash(s2) == want["C2"]
    assert scenegen.sha256_arrays([cam2.R, cam2.t, cam2.C]) == want["C2_camera"]
    assert _hash(scenegen.fd_scene()[0]) == want["FD"]
    _, cams4 = scenegen.c4()
    assert scenegen.sha256_arrays([c.R for c in cams4] + [c.C for c in cams4]) == want["C4_cameras"]


def test_workload_shapes():
    s1, cam1 = scenegen.c1()
    assert s1.n == 10_000 and s1.sh_degree == 0 and s1.sh.shape == (3, 10_000)
    assert (cam1.width, cam1.height) == (256, 256) and abs(cam1.fx - 221.7025) < 1e-3
    s2, cam2 = scenegen.c2()
    assert s2.n == 1_000_000 and s2.sh.shape == (48, 1_000_000)
    assert (cam2.width, cam2.height) == (1920, 1080) and abs(cam2.fx - 1662.768) < 1e-2
    assert np.all(np.abs(cam2.C) <= 3.0)
    low = s2.opacity_logits < -1.0
    assert 0.38 < low.mean() < 0.42  # bimodal opacity: 40 % low mode
    for a in (s2.means, s2.log_scales, s2.quats, s2.opacity_logits, s2.sh):
        assert a.dtype == np.float32 and a.flags.c_contiguous
    assert np.allclose(np.linalg.norm(s2.quats, axis=0), 1.0, atol=1e-5)
    _, cams4 = scenegen.c4()
    res = {(c.width, c.height) for c in cams4}
    assert len(cams4) == 64 and res <= {(512, 512), (1280, 720), (1920, 1080)} and len(res) == 3
    for c in cams4:
        assert abs(np.linalg.norm(c.C) - 3.0) < 1e-5


def test_rotation_matrices_are_orthonormal():
    _, cams4 = scenegen.c4()
    for c in cams4:
        R = c.R.astype(np.float64)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-6)
        assert abs(np.linalg.det(R) - 1) < 1e-5


def test_c3_camera_record():
    with open(os.path.join(os.path.dirname(scenegen.__file__), "c3_camera.json")) as f:
        rec = json.load(f)
    assert 40_000_000 <= rec["pairs"] <= 60_000_000
    assert rec["tried"][-1]["candidate"] == rec["candidate"]
