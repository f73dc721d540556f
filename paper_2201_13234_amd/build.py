"""Builds the device library ``libvtess.so`` (HIP for gfx950) in-tree.

Flags that the bit-exact contract depends on:
  -ffp-contract=off  no fused multiply-add from separate * and +,
  -fno-fast-math     IEEE sqrt and division,
  -packed-fp32-ops   off (the packed FP32 instructions are not used at all).
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvtess.so")
SOURCES = ["label_batch.hip", "label_kernel.hip", "bin_kernels.hip", "nd_kernels.hip", "api.hip"]
# The labelling kernel never sees a NaN (sites are checked by the binning
# pass and a job with bad input is skipped), so min/max need no quieting;
# infinities stay honoured.
EXTRA = {"label_kernel.hip": ["-fno-honor-nans"], "label_batch.hip": ["-fno-honor-nans"]}
ARCH = os.environ.get("VT_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-ffp-contract=off", "-fno-fast-math",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-result",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(src, verbose):
    out = os.path.join(OBJ, src.replace(".hip", ".o"))
    cmd = ["hipcc", *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    warn = [l for l in r.stderr.splitlines()
            if "warning" in l and "packed-fp32-ops" not in l and "not a recognized feature" not in l]
    if warn and verbose:
        print("\n".join(warn), file=sys.stderr)
    return out


def build(verbose=False):
    """Compiles every source and links libvtess.so; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
