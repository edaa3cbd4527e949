"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

* The argument validation (lbm_validate.cpp) with a C++ driver built by g++:
  every rejected parameter, table and geometry, NULL pointers, empty and
  one-byte message buffers, non-finite values.
* The whole library built with the sanitizers on its host code (hipcc with
  -Xarch_host, device code as usual) under a plain-C driver that calls every
  entry point on the paths the host decides alone (NULL handles, invalid
  arguments of the handle calls, the permeability library and the
  capillary-pressure sweep) and the valid calls that reach the device, which
  return LBM_E_DEVICE without a GPU.  Leak checking is on, with the HIP
  runtime's own allocations suppressed."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_sanitize")
CSRC = os.path.join(ROOT, "paper_2512_21696_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(exe, env_extra=None, timeout=300):
    env = dict(os.environ)
    env.update(env_extra or {})
    r = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


def test_validation_under_sanitizers():
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "validate_driver")
        subprocess.run(["g++", "-std=c++17", "-g", "-O1"] + SAN +
                       [os.path.join(HERE, "validate_driver.cpp"),
                        os.path.join(CSRC, "lbm_validate.cpp"), "-o", exe], check=True)
        out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1"})
    assert "all checks passed" in out


@pytest.mark.slow
def test_abi_host_paths_under_sanitizers():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("no ROCm compilers")
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "liblbm_san.so")
        host = []
        for f in SAN:
            host += ["-Xarch_host", f]
        subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                        "-shared", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-Wno-unused-result"] + host +
                       [os.path.join(CSRC, "lbm_runtime.hip"), os.path.join(CSRC, "lbm_validate.cpp"),
                        "-o", lib, "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"],
                       check=True, capture_output=True)
        exe = os.path.join(d, "abi_driver")
        subprocess.run([CLANG, "-std=c11", "-g", "-O1"] + SAN +
                       [os.path.join(HERE, "abi_driver.c"), lib, "-Wl,-rpath," + d,
                        "-Wl,-rpath,/opt/rocm/lib", "-o", exe], check=True)
        supp = os.path.join(d, "lsan.supp")
        with open(supp, "w") as f:
            f.write("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libamd_comgr\nleak:librocprof\n")
        out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1",
                         "LSAN_OPTIONS": "suppressions=" + supp})
    assert "all checks passed" in out
