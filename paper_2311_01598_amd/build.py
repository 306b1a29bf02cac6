"""Build the HIP key-switching library for gfx950 (in-tree): libks.so, and
libks_check.so, the same sources compiled with KS_CHECK_RANGES (every lazy
range and accumulator bound tested where it is used, violations counted on
the device; ks_range_violations reads them)."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libks.so")
OUT_CHECK = os.path.join(HERE, "libks_check.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["numtheory.cpp", "plan.cpp", "api.cpp", "kernels.hip", "rates.hip", "mlp.hip", "noalloc.hip", "ks64.hip",
           "probe.hip"] + ["oc_a%d.hip" % a for a in range(4, 10)]
FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]
VARIANTS = {OUT: (BUILD, []), OUT_CHECK: (os.path.join(BUILD, "check"), ["-DKS_CHECK_RANGES"])}


def _compile(src, bdir, defs, verbose):
    obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = ["hipcc"] + FLAGS + defs + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature; that warning is harmless
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (src, "\n".join(msgs)))
    if msgs and verbose:
        print("\n".join(msgs), flush=True)
    return obj


def build(verbose=False):
    jobs = []
    for out, (bdir, defs) in VARIANTS.items():
        os.makedirs(bdir, exist_ok=True)
        jobs += [(out, src, bdir, defs) for src in SOURCES]
    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(lambda j: (j[0], _compile(j[1], j[2], j[3], verbose)), jobs))
    for out in VARIANTS:
        cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for lib, o in objs if lib == out]
        cmd += ["-o", out + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
