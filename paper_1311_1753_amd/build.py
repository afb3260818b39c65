"""Builds libhipfit.so (gfx950) in-tree with hipcc.

    python -m paper_1311_1753_amd.build        # or build() from Python

Every HIP source is compiled for gfx950 only; the library links the HIP
runtime and nothing else.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build", "hipfit")
LIB = os.path.join(HERE, "libhipfit.so")

SOURCES = ["eval_kernels.hip", "terms_kernels.hip", "full_kernels.hip", "grid_kernels.hip", "gen_kernels.hip", "graph.cpp", "api.cpp",
           "minimiser.cpp", "fit.cpp", "batch.cpp", "noalloc.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          "-Wno-unused-value", "-Wno-unused-result", "-I" + os.path.join(ROOT, "include"),
          "-I/opt/rocm/include"]
DEVICE = ["--offload-arch=gfx950", "-ffp-contract=on", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops"]


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJ, src + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip"] + COMMON + DEVICE + ["-c", path, "-o", obj]
    else:
        cmd = [HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__"] + COMMON + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature; that warning is expected
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines()
            if ln.strip() and "packed-fp32-ops" not in ln]
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (src, " ".join(cmd), "\n".join(msgs)))
    return src, msgs


def build(verbose=False):
    """Compiles every source and links libhipfit.so (always rebuilds)."""
    os.makedirs(OBJ, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        for src, msgs in ex.map(_compile, SOURCES):
            if verbose and msgs:
                print("\n".join(msgs))
    tmp = LIB + ".tmp%d" % os.getpid()
    objs = [os.path.join(OBJ, s + ".o") for s in SOURCES]
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


def clean():
    shutil.rmtree(OBJ, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
