"""Write the stored expected values under tests/golden/.

Only the seeded generators (scenegen) and the CPU oracle are called; nothing
here comes from the GPU library.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenegen  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def scene_hash(scene):
    return scenegen.sha256_arrays([scene.means, scene.log_scales, scene.quats, scene.opacity_logits, scene.sh])


def main():
    out = {}
    s1, _ = scenegen.c1()
    out["C1"] = scene_hash(s1)
    s2, cam2 = scenegen.c2()
    out["C2"] = scene_hash(s2)
    out["C2_camera"] = scenegen.sha256_arrays([cam2.R, cam2.t, cam2.C])
    sfd, _ = scenegen.fd_scene()
    out["FD"] = scene_hash(sfd)
    _, cams4 = scenegen.c4()
    out["C4_cameras"] = scenegen.sha256_arrays([c.R for c in cams4] + [c.C for c in cams4])
    out["C4_resolutions"] = [[c.width, c.height] for c in cams4]
    with open(os.path.join(HERE, "scenegen_sha256.json"), "w") as f:
        json.dump(out, f, indent=1)
    # oracle statistics of the 1M-Gaussian 1080p workload: the counts that fix its algorithmic work
    opts = oracle.Options(sh_degree=3)
    r = oracle.render(s2, cam2, opts)
    p = r["proj"]
    stats = {
        "n": int(s2.n),
        "status_counts": [int(x) for x in (p["status"][:, None] == range(5)).sum(0)],
        "pairs": int(p["tiles_touched"].sum()),
        "evaluations": int(r["n_eval"].sum()),
        "contributions": int(r["n_contrib"].sum()),
        "note": "fp64 oracle forward of the 1M-Gaussian 1920x1080 scene; status order: visible, opacity, near, "
                "degenerate, viewport; evaluations = (pixel, splat) entries inside the splat rectangle visited "
                "before the pixel stops; contributions = those composited",
    }
    with open(os.path.join(HERE, "c2_oracle_stats.json"), "w") as f:
        json.dump(stats, f, indent=1)


if __name__ == "__main__":
    main()
