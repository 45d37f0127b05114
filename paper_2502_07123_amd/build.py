"""Build libmlmc.so (HIP kernels for gfx950 + the C-ABI runtime) in the package
directory with hipcc.

    python -m paper_2502_07123_amd.build         # or build() from Python
    python -m paper_2502_07123_amd.build --probe # also the issue-rate probe executable

Always recompiles (objects go to _build/ next to the package).
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(os.path.dirname(PKG), "_build")
LIB = os.path.join(PKG, "libmlmc.so")
ARCH = "gfx950"

SOURCES = ["kernels.hip", "host_check.hip", "errmodel.hip", "static_entry.hip", "inverse_normal.hip", "engine_kernels.hip", "engine.cpp", "runtime.cpp", "server.cpp",
           "host/prepare.cpp", "host/widths.cpp", "host/choose.cpp"]

FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-Wall",
         "-Wno-unused-function", "-Wno-unused-variable",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _compile(hipcc, src):
    obj = os.path.join(BUILD, src.replace("/", "_") + ".o")
    cmd = [hipcc, "-x", "hip", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (r.stderr or "").splitlines() if noise not in l and "(ignoring feature)" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{err}")
    return obj, err


PROBE_SRC = os.path.join(CSRC, "probe", "issue_rates.hip")
PROBE = os.path.join(PKG, "issue_rates")


def build_probe(hipcc):
    """The VALU issue-rate probe (an executable beside the library)."""
    tmp = PROBE + ".tmp"
    cmd = [hipcc, "-x", "hip", *FLAGS, "-o", tmp, PROBE_SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, PROBE)
    return PROBE


def build(verbose=False, probe=False):
    """The library; with probe, also the issue-rate probe (measurement runs only)."""
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        results = list(ex.map(lambda s: _compile(hipcc, s), SOURCES))
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp,
           *[o for o, _ in results], "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    if probe:
        build_probe(hipcc)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, probe="--probe" in sys.argv))
