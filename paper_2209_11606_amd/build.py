"""Build the HIP library libvorohip.so in-tree with hipcc for gfx950.

python -m paper_2209_11606_amd.build [-v] [--phase-clocks]
--phase-clocks builds libvorohip_phase.so instead: the same library with the
grouped cell kernel's per-phase shader-clock counters (diagnostic slots 16-31).
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvorohip.so")
LIB_PHASE = os.path.join(HERE, "libvorohip_phase.so")
SOURCES = ["binning.hip", "cell3d.hip", "cell3d_group.hip", "cell2d.hip", "weinberg.hip", "peak.hip", "api.cpp"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         # no packed FP32 instructions anywhere in the library
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def build(verbose=False, phase_clocks=False, jobs=None):
    """Compile every source (in parallel) and link the shared library."""
    out = LIB_PHASE if phase_clocks else LIB
    tag = ".phase" if phase_clocks else ""
    defines = ["-DVC_PHASE_CLOCKS"] if phase_clocks else []

    def compile_one(src):
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + tag + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = ["hipcc"] + FLAGS + defines + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd, stderr=subprocess.STDOUT if verbose else None)
        return obj

    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = out + ".tmp"
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, phase_clocks="--phase-clocks" in sys.argv))
