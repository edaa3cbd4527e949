"""Builds the gfx950 shared library liblbm.so in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
# the same library with the device-side index checks (-DLBM_DEBUG)
DEBUG_LIB = os.path.join(HERE, "liblbm_debug.so")
PROBE_LIB = os.path.join(HERE, "libhbmprobe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["lbm_runtime.hip", "lbm_validate.cpp"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]
_ROCTX = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
LIBS = {"liblbm.so": _ROCTX, "liblbm_debug.so": ["-DLBM_DEBUG"] + _ROCTX}


def _compile(sources, out, verbose):
    cmd = ([HIPCC] + FLAGS + [os.path.join(CSRC, s) for s in sources] + ["-o", out + ".tmp"] +
           LIBS.get(os.path.basename(out), []))
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False) -> str:
    """Compiles the method's library, its debug variant and the bandwidth yardstick library."""
    _compile(SOURCES, LIB, verbose)
    _compile(SOURCES, DEBUG_LIB, verbose)
    _compile(["hbm_probe.hip"], PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
