"""Record which seeded camera candidate the 6M-Gaussian 4K workload uses.

The workload asks for 40-60 million (tile, splat) pairs.  This script walks
the seeded candidate list of the shape-scene generator and records the first
candidate whose pair count, computed by the fp64 CPU oracle, lands in that
window.  It writes c3_camera.json next to this file.  Run from the
repository root:  python -m scenegen.pick_c3_camera
"""
import json
import os
import sys
import time

import oracle
import scenegen

LO, HI = 40_000_000, 60_000_000


def main(max_candidates=32):
    scene, cams = scenegen.c3_candidates(count=max_candidates)
    opts = oracle.Options(sh_degree=3)
    tried = []
    for k, cam in enumerate(cams):
        t = time.time()
        m = oracle.pair_count(scene, cam, opts)
        tried.append({"candidate": k, "pairs": m})
        print(f"candidate {k}: M = {m:,} ({time.time() - t:.1f} s)", flush=True)
        if LO <= m <= HI:
            out = {"candidate": k, "pairs": m, "window": [LO, HI], "tried": tried,
                   "note": "first seeded candidate whose oracle pair count lies in the window"}
            path = os.path.join(os.path.dirname(__file__), "c3_camera.json")
            with open(path, "w") as f:
                json.dump(out, f, indent=1)
            print("wrote", path)
            return 0
    print("no candidate in the window", file=sys.stderr)
    return 1


if __name__ == "__main__":
    sys.exit(main())
