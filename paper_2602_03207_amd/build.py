"""Build libwebsplat.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2602_03207_amd.build   (or via __graft_entry__.build()).
"""
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwebsplat.so")
SOURCES = ["api.hip", "preprocess.hip", "sort.hip", "render.hip", "backward.hip", "loss.hip", "noalloc.hip"]
ARCH = "gfx950"


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def compile_flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
        # never emit packed fp32 arithmetic (v_pk_*_f32)
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-munsafe-fp-atomics",
        # atomics stay as written: the optimizer's wave-level rewrite of atomics to one (uniform) address
        # adds a read-lane loop and lane counting in front of adds that a single lane makes
        "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
        f"-I{os.path.join(HERE, '..', 'include')}",
    ]


def build(verbose=True, jobs=8):
    """Compile every .hip source to an object, then link the shared library."""
    t0 = time.time()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc(), *compile_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = False
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"--- {src}\n{out}\n")
        elif verbose:
            lines = [l for l in out.splitlines() if l.strip() and "packed-fp32-ops" not in l
                     and "warning generated" not in l and "warnings generated" not in l]
            if lines:
                sys.stderr.write(f"--- {src} (warnings)\n" + "\n".join(lines) + "\n")
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f} s")
    return LIB


if __name__ == "__main__":
    build()
