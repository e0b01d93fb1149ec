"""Builds libdpo.so (hipcc, gfx950) from the traversal sources in csrc/, and
libdpo_calib.so (the roofline calibration kernels, measurement only), in the
package folder."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdpo.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("dpo_kernels.hip", "dpo_host.hip")]
CALIB_LIB = os.path.join(HERE, "libdpo_calib.so")
CALIB_SOURCES = [os.path.join(HERE, "csrc", "dpo_calib.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # no packed-FP32 instructions in any HIP code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]


def _hipcc(sources, lib, verbose):
    tmp = lib + ".tmp"
    cmd = [HIPCC, *FLAGS, *sources, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(lib)}")
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    _hipcc(CALIB_SOURCES, CALIB_LIB, verbose)
    return _hipcc(SOURCES, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
